// FP64 CPU oracle for the short-characteristics radiation transport solve of
// arXiv 2107.08145 (MURaM), section "Summary of the Radiation Transport Solver"
// and the RTS core loop figure (per ray: interpolate, then iterate
// integrate / write buffer / exchange, then flux).
//
// TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
// HIP library is checked against.  Only the tests, the smoke check and the
// benchmark's CPU-baseline leg may load it.  It shares no code with the HIP
// path (no headers, helpers, tables or generators); it sees only the problem
// statement as plain arrays.
//
// What is computed (the readings of the paper's unstated details are listed
// in the design notes of the repository):
//   * chi_b = kappa_b * rho, the extinction per unit length.
//   * Per ray (unit direction mu, weight w): ds = min over axes d with
//     mu_d != 0 of delta_d / |mu_d|; the arg-min is the dominant axis (ties go
//     to z, then y, then x).  Each cell's upwind point lies ds back along the
//     ray, in the previous grid plane along the dominant axis, between the
//     four cells offset by 0 / -sign(mu_e) along the two in-plane axes e, at
//     fractions f_e = ds |mu_e| / delta_e ("up to four" upwind points in the
//     wavefront-dependency figure).  I, S and chi there are bilinear in those
//     four cells.
//   * Optical depth of the segment: trapezoid, dtau = ds/2 (chi_p + chi_u).
//   * Formal solution with S linear in optical depth between u and p,
//     integrated exactly against exp(-t):
//        I_p = e I_u + w0 S_p + w1 S_u,  e = exp(-x),
//        w0 = (x - 1 + e)/x,  w1 = (1 - e (1 + x))/x,  x = dtau,
//     with the power series below x = 0.5 (where the closed forms cancel).
//   * Boundaries: x and y periodic; rays with mu_z > 0 start from the bottom
//     layer k = 0 (I = S, or a fixed I), rays with mu_z < 0 from the top layer
//     k = nz-1 (I = 0, or I = S).  These layers are set, not integrated.
//   * Periodic boundary iteration (the paper's "3 to 4 iterations" of
//     boundary intensities, exchanged through buffers): a ray whose dominant
//     axis is x or y reads its first plane's upwind intensities from a ghost
//     plane.  The ghost starts at I = S (boundary-layer cells at their boundary
//     value) and is overwritten with the last swept plane after each of the
//     n_iter sweeps.  Rays with a z dominant axis need no ghost: one sweep.
//   * Flux: J_b = sum_r w_r I_r after the last sweep; I_top = I in the top
//     layer for mu_z > 0 rays; Q = sum_b qweight_b 4 pi chi_b (J_b - S_b).
//   * Tolerance-driven boundary iteration (the paper iterates the boundary
//     intensities until their error is within a prescribed tolerance): with
//     tol > 0, the rays of one band that share an x or y dominant axis and its
//     direction (a group swept together) repeat their sweeps until the largest
//     change of their outflow-plane intensities between successive sweeps is
//     at most tol times the largest outflow-plane intensity (the first sweep
//     compares with the initial ghost), n_iter sweeps at most.
//   * Radiative flux vector (the flux step computes mean intensity and fluxes
//     from the same rays): F = sum_b qweight_b 4 pi sum_r w_r mu_r I_r, and the
//     heating -div F by central differences (periodic in x and y; second-order
//     one-sided differences in the bottom and top layers).
//   * Adjoint: the reverse-mode derivative of the above (downwind to upwind,
//     last sweep first, ghost sensitivities carried into the previous sweep).
//   * Scattering (the paper's Gauss-Seidel scheme for strongly scattering
//     media): S = (1 - eps) J + eps B updated at every point as the rays are
//     integrated, the new value feeding the next point along the ray.
//   * Subdomain decomposition (the paper's domain-decomposed RTS): blocks of
//     the grid iterate with the intensities their upwind neighbours produced
//     in the previous iteration (block Jacobi across blocks, exact sweeps
//     inside a block), n_iter iterations or until a global tolerance.
//
// Build: g++ -O2 -std=c++17 -fPIC -shared -ffp-contract=off -fno-fast-math -fopenmp
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using cplx = std::complex<double>;

inline double re(double v) { return v; }
inline double re(const cplx& v) { return v.real(); }

constexpr double kPi = 3.14159265358979323846;
constexpr double kSeriesBelow = 0.5;  // closed forms lose < 2e-15 relative above this

// Problem statement.
struct Desc {
  int n[3];          // nx, ny, nz
  double d[3];       // dx, dy, dz
  int nb, nr;        // bands, rays
  const double* mu;  // [nr][3]
  const double* w;   // [nr]
  const double* qw;  // [nb]
  int bot, top;      // 0: thermal bottom / zero top, 1: fixed bottom / thermal top
  double ibot;
  int n_iter;
  double tol = 0.0;  // > 0: sweeps of a group stop at this relative change (n_iter at most)
  // warm start: the initial ghost planes (I) of the x and y dominant rays, and
  // their final ones, [nb][nr][nz][max(nx, ny)] (row k, horizontal index j)
  const double* gin = nullptr;
  double* gout = nullptr;
  int64_t cells() const { return (int64_t)n[0] * n[1] * n[2]; }
  int64_t at(int i, int j, int k) const { return ((int64_t)k * n[1] + j) * n[0] + i; }
};

// Linear-source weights (e, w0, w1) for optical depth x.
template <class T>
struct Wts { T e, w0, w1; };

template <class T>
Wts<T> weights(const T& x) {
  Wts<T> r;
  r.e = std::exp(-x);
  if (re(x) < kSeriesBelow) {
    // w0 = sum_{n>=2} (-1)^n x^(n-1)/n!,  w1 = sum_{n>=2} (-1)^n (n-1) x^(n-1)/n!
    T term = x / 2.0;
    T w0 = 0.0, w1 = 0.0;
    for (int n = 2; n <= 22; ++n) {
      w0 += term;
      w1 += double(n - 1) * term;
      term *= -x / double(n + 1);
    }
    r.w0 = w0;
    r.w1 = w1;
  } else {
    r.w0 = (x - 1.0 + r.e) / x;
    r.w1 = (1.0 - r.e * (1.0 + x)) / x;
  }
  return r;
}

// w1 / x, which is dw0/dx; dw1/dx = e - w1/x.
double w1_over_x(double x, double e) {
  if (x < kSeriesBelow) {
    // sum_{n>=2} (-1)^n (n-1) x^(n-2) / n!
    double term = 0.5, s = 0.0;
    for (int n = 2; n <= 23; ++n) {
      s += double(n - 1) * term;
      term *= -x / double(n + 1);
    }
    return s;
  }
  return (1.0 - e * (1.0 + x)) / (x * x);
}

// Per-ray geometry.
struct Ray {
  int axis, sa;      // dominant axis and its sign
  int ea, eb;        // in-plane axes, ea < eb
  int sea, seb;      // signs along them
  double fa, fb;     // upwind fractions along them
  double ds;         // path length to the upwind plane
  bool up;           // mu_z > 0
};

bool make_ray(const Desc& D, const double* mu, Ray& r) {
  if (mu[2] == 0.0) return false;
  double best = INFINITY;
  r.axis = -1;
  for (int d = 0; d < 3; ++d) {
    if (mu[d] == 0.0) continue;
    double s = D.d[d] / std::fabs(mu[d]);
    if (s <= best) { best = s; r.axis = d; }  // later axis wins ties: z, then y, then x
  }
  r.ds = best;
  r.sa = mu[r.axis] > 0 ? 1 : -1;
  int e[2], m = 0;
  for (int d = 0; d < 3; ++d) if (d != r.axis) e[m++] = d;
  r.ea = e[0]; r.eb = e[1];
  r.sea = mu[r.ea] >= 0 ? 1 : -1;
  r.seb = mu[r.eb] >= 0 ? 1 : -1;
  r.fa = r.ds * std::fabs(mu[r.ea]) / D.d[r.ea];
  r.fb = r.ds * std::fabs(mu[r.eb]) / D.d[r.eb];
  r.up = mu[2] > 0;
  return true;
}

inline int wrap(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

// Boundary-layer intensity for a cell with source function s.
template <class T>
T bc_value(const Desc& D, const Ray& r, const T& s) {
  if (r.up) return D.bot == 0 ? s : T(D.ibot);
  return D.top == 0 ? T(0.0) : s;
}

inline bool is_bc_layer(const Desc& D, const Ray& r, int k) {
  return r.up ? (k == 0) : (k == D.n[2] - 1);
}

// The sweeps of one ray of one band, I overwritten: set-up (boundary layer
// and initial ghost plane), then one sweep per call of sweep().
template <class T>
struct RaySweeper {
  const Desc& D;
  const Ray& r;
  const T* chi;
  const T* S;
  T* I;
  int nt;
  int na, nA, nB, q_first, q_last;
  bool periodic;
  double b00, b10, b01, b11;
  std::vector<T> ghost;

  int64_t cell(int q, int a, int b) const {
    int c[3];
    c[r.axis] = q; c[r.ea] = a; c[r.eb] = b;
    return D.at(c[0], c[1], c[2]);
  }
  int kz(int q, int a, int b) const {
    int c[3];
    c[r.axis] = q; c[r.ea] = a; c[r.eb] = b;
    return c[2];
  }

  // warm: this ray's initial ghost plane [nz][max(nx, ny)] or null (I = S)
  RaySweeper(const Desc& D_, const Ray& r_, const T* chi_, const T* S_, T* I_, int nt_,
             const double* warm = nullptr)
      : D(D_), r(r_), chi(chi_), S(S_), I(I_), nt(nt_) {
    na = D.n[r.axis]; nA = D.n[r.ea]; nB = D.n[r.eb];
    periodic = r.axis != 2;
    b00 = (1 - r.fa) * (1 - r.fb); b10 = r.fa * (1 - r.fb);
    b01 = (1 - r.fa) * r.fb; b11 = r.fa * r.fb;
    q_first = r.sa > 0 ? 0 : na - 1;
    q_last = r.sa > 0 ? na - 1 : 0;
    // Boundary layer: set, not integrated.
    for (int q = 0; q < na; ++q)
      for (int a = 0; a < nA; ++a)
        for (int b = 0; b < nB; ++b)
          if (is_bc_layer(D, r, kz(q, a, b))) {
            int64_t p = cell(q, a, b);
            I[p] = bc_value(D, r, S[p]);
          }
    // Ghost plane for periodic sweeps: I = S of the wrapped upwind plane, or
    // the given warm-start intensities (the in-plane axes are the horizontal
    // one, a, and z, b); boundary-layer cells at their boundary value.
    if (periodic) {
      const int M = std::max(D.n[0], D.n[1]);
      ghost.resize((size_t)nA * nB);
      for (int a = 0; a < nA; ++a)
        for (int b = 0; b < nB; ++b) {
          int64_t p = cell(q_last, a, b);
          ghost[(size_t)a * nB + b] =
              is_bc_layer(D, r, kz(q_last, a, b)) ? bc_value(D, r, S[p])
              : warm                              ? T(warm[(size_t)b * M + a])
                                                  : S[p];
        }
    }
  }

  // The current ghost plane (the last sweep's outflow plane) into out [nz][max(nx, ny)].
  void save_ghost(double* out) const {
    if (!periodic || !out) return;
    const int M = std::max(D.n[0], D.n[1]);
    for (int a = 0; a < nA; ++a)
      for (int b = 0; b < nB; ++b) out[(size_t)b * M + a] = re(ghost[(size_t)a * nB + b]);
  }

  // One sweep; the outflow plane becomes the next sweep's ghost.  Returns the
  // largest change of the ghost plane's intensities and its largest intensity
  // (periodic rays; zeros otherwise).
  std::pair<double, double> sweep() {
    // z-dominant rays start one plane in: their first plane is the boundary layer.
    for (int t = periodic ? 0 : 1; t < na; ++t) {
      const int q = q_first + r.sa * t;
      const int qu = wrap(q - r.sa, na);
      const bool from_ghost = periodic && t == 0;
#pragma omp parallel for collapse(2) num_threads(nt) schedule(static)
      for (int a = 0; a < nA; ++a)
        for (int b = 0; b < nB; ++b) {
          if (is_bc_layer(D, r, kz(q, a, b))) continue;
          const int64_t p = cell(q, a, b);
          // upwind corners (in-plane z never leaves the grid for a non-boundary cell)
          const int a1 = r.ea == 2 ? a - r.sea : wrap(a - r.sea, nA);
          const int b1 = r.eb == 2 ? b - r.seb : wrap(b - r.seb, nB);
          const int64_t u00 = cell(qu, a, b), u10 = cell(qu, a1, b);
          const int64_t u01 = cell(qu, a, b1), u11 = cell(qu, a1, b1);
          T i00, i10, i01, i11;
          if (from_ghost) {
            i00 = ghost[(size_t)a * nB + b];  i10 = ghost[(size_t)a1 * nB + b];
            i01 = ghost[(size_t)a * nB + b1]; i11 = ghost[(size_t)a1 * nB + b1];
          } else {
            i00 = I[u00]; i10 = I[u10]; i01 = I[u01]; i11 = I[u11];
          }
          const T iu = b00 * i00 + b10 * i10 + b01 * i01 + b11 * i11;
          const T su = b00 * S[u00] + b10 * S[u10] + b01 * S[u01] + b11 * S[u11];
          const T cu = b00 * chi[u00] + b10 * chi[u10] + b01 * chi[u01] + b11 * chi[u11];
          const T x = 0.5 * r.ds * (chi[p] + cu);
          const Wts<T> wt = weights(x);
          I[p] = wt.e * iu + wt.w0 * S[p] + wt.w1 * su;
        }
    }
    double diff = 0.0, scale = 0.0;
    if (periodic) {  // exchange: the outflow plane becomes the next sweep's ghost
      for (int a = 0; a < nA; ++a)
        for (int b = 0; b < nB; ++b) {
          const T v = I[cell(q_last, a, b)];
          T& g = ghost[(size_t)a * nB + b];
          diff = std::max(diff, std::fabs(re(v) - re(g)));
          scale = std::max(scale, std::fabs(re(v)));
          g = v;
        }
    }
    return {diff, scale};
  }
};

// One ray of one band: n_iter sweeps (1 for z-dominant rays), I overwritten.
// If `store` is given, the intensities after every sweep are appended to it.
template <class T>
void solve_ray(const Desc& D, const Ray& r, const T* chi, const T* S, T* I,
               std::vector<std::vector<T>>* store, int nt, const double* warm = nullptr,
               double* gout = nullptr) {
  RaySweeper<T> w(D, r, chi, S, I, nt, warm);
  const int sweeps = w.periodic ? D.n_iter : 1;
  for (int sweep = 0; sweep < sweeps; ++sweep) {
    w.sweep();
    if (store) store->emplace_back(I, I + D.cells());
  }
  w.save_ghost(gout);
}

template <class T>
int forward(const Desc& D, const T* chi, const T* S, T* Q, T* J, T* Itop, int nt,
            std::vector<std::vector<T>>* store, std::vector<T>* Jall, T* F = nullptr,
            int* sweeps_used = nullptr) {
  const int64_t N = D.cells();
  std::vector<Ray> rays(D.nr);
  for (int r = 0; r < D.nr; ++r)
    if (!make_ray(D, D.mu + 3 * r, rays[r])) return -1;
  for (int64_t p = 0; p < N; ++p) Q[p] = 0.0;
  if (F)
    for (int64_t p = 0; p < 3 * N; ++p) F[p] = 0.0;
  std::vector<T> I(N), Jb(N);
  const int64_t plane = (int64_t)D.n[0] * D.n[1];
  int nup = 0;
  for (int r = 0; r < D.nr; ++r) nup += rays[r].up;
  std::vector<std::vector<T>> Iall;
  if (D.tol > 0) Iall.assign(D.nr, std::vector<T>(N));
  const int64_t gstride = (int64_t)D.n[2] * std::max(D.n[0], D.n[1]);  // one ray's ghost
  auto gin_of = [&](int b, int r) { return D.gin ? D.gin + ((int64_t)b * D.nr + r) * gstride : nullptr; };
  auto gout_of = [&](int b, int r) { return D.gout ? D.gout + ((int64_t)b * D.nr + r) * gstride : nullptr; };
  for (int b = 0; b < D.nb; ++b) {
    const T* chib = chi + b * N;
    const T* Sb = S + b * N;
    for (int64_t p = 0; p < N; ++p) Jb[p] = 0.0;
    if (D.tol > 0) {
      // every ray first; groups (x or y dominant axis, direction) in lock step
      std::vector<char> done(D.nr, 0);
      for (int r0 = 0; r0 < D.nr; ++r0) {
        if (done[r0]) continue;
        std::vector<int> grp;
        for (int r = r0; r < D.nr; ++r)
          if (!done[r] && rays[r].axis == rays[r0].axis && rays[r].sa == rays[r0].sa) grp.push_back(r);
        std::vector<RaySweeper<T>> ws;
        for (int r : grp) {
          done[r] = 1;
          ws.emplace_back(D, rays[r], chib, Sb, Iall[r].data(), nt, gin_of(b, r));
        }
        const int max_sweeps = rays[r0].axis != 2 ? D.n_iter : 1;
        int used = 0;
        for (int sweep = 0; sweep < max_sweeps; ++sweep) {
          double diff = 0.0, scale = 0.0;
          for (auto& w : ws) {
            const auto ds = w.sweep();
            diff = std::max(diff, ds.first);
            scale = std::max(scale, ds.second);
          }
          used = sweep + 1;
          if (rays[r0].axis != 2 && diff <= D.tol * scale) break;
        }
        if (sweeps_used)
          for (int r : grp) sweeps_used[b * D.nr + r] = used;
        for (size_t k = 0; k < grp.size(); ++k) ws[k].save_ghost(gout_of(b, grp[k]));
      }
    }
    int ru = 0;
    for (int r = 0; r < D.nr; ++r) {
      if (D.tol > 0) std::copy(Iall[r].begin(), Iall[r].end(), I.begin());
      else solve_ray(D, rays[r], chib, Sb, I.data(), store, nt, gin_of(b, r), gout_of(b, r));
      for (int64_t p = 0; p < N; ++p) Jb[p] += D.w[r] * I[p];
      if (F)
        for (int k = 0; k < 3; ++k) {
          const double fk = 4.0 * kPi * D.qw[b] * D.w[r] * D.mu[3 * r + k];
          for (int64_t p = 0; p < N; ++p) F[k * N + p] += fk * I[p];
        }
      if (rays[r].up) {
        if (Itop) {
          T* dst = Itop + ((int64_t)b * nup + ru) * plane;
          for (int64_t p = 0; p < plane; ++p) dst[p] = I[(int64_t)(D.n[2] - 1) * plane + p];
        }
        ++ru;
      }
    }
    const double qf = 4.0 * kPi * D.qw[b];
    for (int64_t p = 0; p < N; ++p) Q[p] += qf * chib[p] * (Jb[p] - Sb[p]);
    if (J) std::memcpy(J + b * N, Jb.data(), sizeof(T) * N);
    if (Jall) Jall->insert(Jall->end(), Jb.begin(), Jb.end());
  }
  return 0;
}

// Second oracle mode: the same discrete scheme written for D = I - S.  With
// e + w0 + w1 = 1 and the bilinear interpolation being linear, the linear-
// source update becomes D_p = e B(D) + c (B(S) - S_p), c = (1 - e)/x.  This is
// a separate implementation of every step (boundary values, ghost plane,
// sweep, flux step) so that agreement with forward() checks the identity.
//   Boundary layers: D = I_bc - S (0 for a thermal bottom, i_bot - S for a
//   fixed one, -S for a zero top, 0 for a thermal top); initial ghost D = 0
//   off the boundary layer; J_b = (sum_r w_r) S_b + sum_r w_r D_r, Q from
//   J_b - S_b = (sum_r w_r - 1) S_b + sum_r w_r D_r; I_top = S + D.
double c_weight(double x) {
  if (x < 0.1) {  // sum_{n>=0} (-x)^n / (n+1)!, through n = 12
    double term = 1.0, s = 0.0;
    for (int n = 0; n <= 12; ++n) {
      s += term;
      term *= -x / double(n + 2);
    }
    return s;
  }
  return -std::expm1(-x) / x;
}

int forward_dform(const Desc& D, const double* chi, const double* S, double* Q, double* J,
                  double* Itop) {
  const int64_t N = D.cells();
  const int64_t plane = (int64_t)D.n[0] * D.n[1];
  std::vector<Ray> rays(D.nr);
  for (int r = 0; r < D.nr; ++r)
    if (!make_ray(D, D.mu + 3 * r, rays[r])) return -1;
  double wsum = 0.0;
  for (int r = 0; r < D.nr; ++r) wsum += D.w[r];
  int nup = 0;
  for (int r = 0; r < D.nr; ++r) nup += rays[r].up;
  for (int64_t p = 0; p < N; ++p) Q[p] = 0.0;
  std::vector<double> Dv(N), dJ(N), ghost;
  for (int b = 0; b < D.nb; ++b) {
    const double* cb = chi + b * N;
    const double* sb = S + b * N;
    for (int64_t p = 0; p < N; ++p) dJ[p] = 0.0;
    int ru = 0;
    for (int r = 0; r < D.nr; ++r) {
      const Ray& R = rays[r];
      const int na = D.n[R.axis], nA = D.n[R.ea], nB = D.n[R.eb];
      const bool periodic = R.axis != 2;
      auto cell = [&](int q, int a, int bb) {
        int c[3];
        c[R.axis] = q; c[R.ea] = a; c[R.eb] = bb;
        return D.at(c[0], c[1], c[2]);
      };
      auto bc_layer = [&](int64_t p) {
        const int k = (int)(p / plane);
        return R.up ? k == 0 : k == D.n[2] - 1;
      };
      auto bc_d = [&](int64_t p) {
        if (R.up) return D.bot == 0 ? 0.0 : D.ibot - sb[p];
        return D.top == 0 ? -sb[p] : 0.0;
      };
      for (int64_t p = 0; p < N; ++p) Dv[p] = bc_layer(p) ? bc_d(p) : 0.0;
      const int q_first = R.sa > 0 ? 0 : na - 1, q_last = R.sa > 0 ? na - 1 : 0;
      if (periodic) {
        ghost.assign((size_t)nA * nB, 0.0);
        for (int a = 0; a < nA; ++a)
          for (int bb = 0; bb < nB; ++bb) {
            const int64_t p = cell(q_last, a, bb);
            if (bc_layer(p)) ghost[(size_t)a * nB + bb] = bc_d(p);
          }
      }
      const double w00 = (1 - R.fa) * (1 - R.fb), w10 = R.fa * (1 - R.fb);
      const double w01 = (1 - R.fa) * R.fb, w11 = R.fa * R.fb;
      const int sweeps = periodic ? D.n_iter : 1;
      for (int it = 0; it < sweeps; ++it) {
        for (int t = periodic ? 0 : 1; t < na; ++t) {
          const int q = q_first + R.sa * t;
          const int qu = wrap(q - R.sa, na);
          for (int a = 0; a < nA; ++a)
            for (int bb = 0; bb < nB; ++bb) {
              const int64_t p = cell(q, a, bb);
              if (bc_layer(p)) continue;
              const int a1 = R.ea == 2 ? a - R.sea : wrap(a - R.sea, nA);
              const int b1 = R.eb == 2 ? bb - R.seb : wrap(bb - R.seb, nB);
              const int64_t u[4] = {cell(qu, a, bb), cell(qu, a1, bb), cell(qu, a, b1),
                                    cell(qu, a1, b1)};
              double du[4];
              if (periodic && t == 0) {
                du[0] = ghost[(size_t)a * nB + bb];
                du[1] = ghost[(size_t)a1 * nB + bb];
                du[2] = ghost[(size_t)a * nB + b1];
                du[3] = ghost[(size_t)a1 * nB + b1];
              } else {
                for (int m = 0; m < 4; ++m) du[m] = Dv[u[m]];
              }
              const double bd = w00 * du[0] + w10 * du[1] + w01 * du[2] + w11 * du[3];
              const double bs = w00 * sb[u[0]] + w10 * sb[u[1]] + w01 * sb[u[2]] + w11 * sb[u[3]];
              const double bx = w00 * cb[u[0]] + w10 * cb[u[1]] + w01 * cb[u[2]] + w11 * cb[u[3]];
              const double x = 0.5 * R.ds * (cb[p] + bx);
              Dv[p] = std::exp(-x) * bd + c_weight(x) * (bs - sb[p]);
            }
        }
        if (periodic)
          for (int a = 0; a < nA; ++a)
            for (int bb = 0; bb < nB; ++bb) ghost[(size_t)a * nB + bb] = Dv[cell(q_last, a, bb)];
      }
      for (int64_t p = 0; p < N; ++p) dJ[p] += D.w[r] * Dv[p];
      if (R.up) {
        if (Itop) {
          double* dst = Itop + ((int64_t)b * nup + ru) * plane;
          const int64_t top = (int64_t)(D.n[2] - 1) * plane;
          for (int64_t p = 0; p < plane; ++p) dst[p] = sb[top + p] + Dv[top + p];
        }
        ++ru;
      }
    }
    const double qf = 4.0 * kPi * D.qw[b];
    for (int64_t p = 0; p < N; ++p) {
      const double djs = (wsum - 1.0) * sb[p] + dJ[p];
      Q[p] += qf * cb[p] * djs;
      if (J) J[b * N + p] = sb[p] + djs;
    }
  }
  return 0;
}

// ---------------------------------------------------------------------------
// Scattering with Gauss-Seidel source updates along the rays.  In a strongly
// scattering medium the source function depends on the radiation field,
// S = (1 - eps) J + eps B (eps: photon destruction probability, B: thermal
// source).  The paper proposes the Gauss-Seidel scheme of Trujillo Bueno &
// Fabiani Bendicho (1995): as a ray is integrated, the source function of
// each point is updated at once and the new value is used for the next point
// along the ray, which merges interpolation and integration.  As in that
// scheme, the rays of the other directions are first integrated with the
// current source function, so that the update at a point sees its complete
// mean intensity, and the update is a local Newton step with the diagonal of
// the transfer operator.  Reading (per band):
//   * Local operator: L(p) = sum_r w_r dI_r(p)/dS_p over every ray, the weight
//     of S_p in the intensities at p itself: w0 of the ray's linear-source
//     step at p (1 for a boundary cell of a ray whose boundary value is S, 0
//     for the others).
//   * S starts at B; every group of rays sharing the dominant axis and its
//     direction (the rays swept together) holds its contribution P_g =
//     sum_{r in g} w_r I_r to J, initially (sum_{r in g} w_r) S, and
//     J = sum_g P_g.
//   * One Gauss-Seidel iteration sweeps the groups in order of first
//     appearance, each with its laps (n_iter for x or y dominant axes, from
//     the ghost plane I = S of the current S, 1 for z).  At every cell p of a
//     plane, each ray of the group takes the linear-source step of the plain
//     solve with the current S (upwind values from the cells already
//     updated), or its boundary value.  The laps before the last iterate the
//     periodic boundary intensities only.  In the last lap, at every cell,
//     P_new = sum_{r in g} w_r I_r and J_p += P_new - P_g(p), P_g(p) = P_new;
//     in the last lap of the last group, before that, the update:
//       J' = J_p + P_new - P_g(p),
//       dS = ((1 - eps_p) J' + eps_p B_p - S_p) / (1 - (1 - eps_p) L(p)),
//       S_p += dS,  I_r += (dI_r/dS_p) dS for the group's rays (so that the
//       next points along the rays integrate from the new source function),
//     with P_new taken from the corrected intensities.
//     A fixed point has dS = 0: S = (1 - eps) J[S] + eps B with J[S] the
//     plain solve's mean intensity.
//   * After n_gs iterations: S, J, Q = sum_b qw_b 4 pi chi_b (J_b - S_b), and
//     I_top from the last sweep of each upward ray.
// With eps = 1 every dS is B - S = 0: S stays B and the sweeps are those of
// forward() on S = B.

// w0 of ray r's step at every cell (dI/dS_p; boundary cells: 1 if their value
// is S, else 0), from chi alone.
void local_weights(const Desc& D, const Ray& r, const double* chi, double* out) {
  const int na = D.n[r.axis], nA = D.n[r.ea], nB = D.n[r.eb];
  const int64_t plane = (int64_t)D.n[0] * D.n[1];
  auto cell = [&](int q, int a, int bb) {
    int c[3];
    c[r.axis] = q; c[r.ea] = a; c[r.eb] = bb;
    return D.at(c[0], c[1], c[2]);
  };
  const double b00 = (1 - r.fa) * (1 - r.fb), b10 = r.fa * (1 - r.fb);
  const double b01 = (1 - r.fa) * r.fb, b11 = r.fa * r.fb;
  for (int q = 0; q < na; ++q) {
    const int qu = wrap(q - r.sa, na);
    for (int a = 0; a < nA; ++a)
      for (int bb = 0; bb < nB; ++bb) {
        const int64_t p = cell(q, a, bb);
        if (is_bc_layer(D, r, (int)(p / plane))) {
          out[p] = r.up ? (D.bot == 0 ? 1.0 : 0.0) : (D.top == 0 ? 0.0 : 1.0);
          continue;
        }
        const int a1 = r.ea == 2 ? a - r.sea : wrap(a - r.sea, nA);
        const int b1 = r.eb == 2 ? bb - r.seb : wrap(bb - r.seb, nB);
        const double cu = b00 * chi[cell(qu, a, bb)] + b10 * chi[cell(qu, a1, bb)] +
                          b01 * chi[cell(qu, a, b1)] + b11 * chi[cell(qu, a1, b1)];
        out[p] = weights(0.5 * r.ds * (chi[p] + cu)).w0;
      }
  }
}

int forward_gs(const Desc& D, const double* chi, const double* Bsrc, const double* eps,
               int n_gs, double* Q, double* J, double* Itop, double* Sout) {
  const int64_t N = D.cells();
  const int64_t plane = (int64_t)D.n[0] * D.n[1];
  std::vector<Ray> rays(D.nr);
  for (int r = 0; r < D.nr; ++r)
    if (!make_ray(D, D.mu + 3 * r, rays[r])) return -1;
  // groups: (dominant axis, direction) in order of first appearance, rays in order
  std::vector<std::vector<int>> groups;
  for (int r = 0; r < D.nr; ++r) {
    bool placed = false;
    for (auto& g : groups)
      if (rays[g[0]].axis == rays[r].axis && rays[g[0]].sa == rays[r].sa) {
        g.push_back(r);
        placed = true;
        break;
      }
    if (!placed) groups.push_back({r});
  }
  const size_t G = groups.size();
  int nup = 0;
  for (int r = 0; r < D.nr; ++r) nup += rays[r].up;
  for (int64_t p = 0; p < N; ++p) Q[p] = 0.0;
  std::vector<double> S(N), Jb(N), P(G * N), Lop(N), W0((size_t)D.nr * N);
  std::vector<std::vector<double>> I, ghost;
  for (int b = 0; b < D.nb; ++b) {
    const double* cb = chi + b * N;
    const double* Bb = Bsrc + b * N;
    const double* eb = eps + b * N;
    for (int r = 0; r < D.nr; ++r) local_weights(D, rays[r], cb, W0.data() + (size_t)r * N);
    for (int64_t p = 0; p < N; ++p) {
      double l = 0.0;
      for (int r = 0; r < D.nr; ++r) l += D.w[r] * W0[(size_t)r * N + p];
      Lop[p] = l;
      S[p] = Bb[p];
      Jb[p] = 0.0;
    }
    for (size_t g = 0; g < G; ++g) {
      double wg = 0.0;
      for (int r : groups[g]) wg += D.w[r];
      for (int64_t p = 0; p < N; ++p) {
        P[g * N + p] = wg * S[p];
        Jb[p] += P[g * N + p];
      }
    }
    for (int it = 0; it < n_gs; ++it) {
      for (size_t g = 0; g < G; ++g) {
        const std::vector<int>& rg = groups[g];
        const Ray& R0 = rays[rg[0]];
        const int na = D.n[R0.axis], nA = D.n[R0.ea], nB = D.n[R0.eb];
        const bool periodic = R0.axis != 2;
        const int laps = periodic ? D.n_iter : 1;
        const int q_first = R0.sa > 0 ? 0 : na - 1, q_last = R0.sa > 0 ? na - 1 : 0;
        auto cell = [&](int q, int a, int bb) {
          int c[3];
          c[R0.axis] = q; c[R0.ea] = a; c[R0.eb] = bb;
          return D.at(c[0], c[1], c[2]);
        };
        I.assign(rg.size(), std::vector<double>(N, 0.0));
        ghost.assign(rg.size(), std::vector<double>((size_t)nA * nB, 0.0));
        if (periodic)  // the ghost plane: I = S of the current S (boundary layer at its value)
          for (size_t k = 0; k < rg.size(); ++k)
            for (int a = 0; a < nA; ++a)
              for (int bb = 0; bb < nB; ++bb) {
                const int64_t p = cell(q_last, a, bb);
                const int kz = (int)(p / plane);
                ghost[k][(size_t)a * nB + bb] =
                    is_bc_layer(D, rays[rg[k]], kz) ? bc_value(D, rays[rg[k]], S[p]) : S[p];
              }
        for (int lap = 0; lap < laps; ++lap) {
          const bool update = lap == laps - 1 && g == G - 1;
          for (int t = 0; t < na; ++t) {
            const int q = q_first + R0.sa * t;
            const int qu = wrap(q - R0.sa, na);
            for (int a = 0; a < nA; ++a)
              for (int bb = 0; bb < nB; ++bb) {
                const int64_t p = cell(q, a, bb);
                const int kz = (int)(p / plane);
                double pn = 0.0;
                for (size_t k = 0; k < rg.size(); ++k) {
                  const Ray& r = rays[rg[k]];
                  double v;
                  if (is_bc_layer(D, r, kz)) {
                    v = bc_value(D, r, S[p]);
                  } else {
                    const int a1 = r.ea == 2 ? a - r.sea : wrap(a - r.sea, nA);
                    const int b1 = r.eb == 2 ? bb - r.seb : wrap(bb - r.seb, nB);
                    const int64_t u00 = cell(qu, a, bb), u10 = cell(qu, a1, bb);
                    const int64_t u01 = cell(qu, a, b1), u11 = cell(qu, a1, b1);
                    double i00, i10, i01, i11;
                    if (periodic && t == 0) {
                      const std::vector<double>& gh = ghost[k];
                      i00 = gh[(size_t)a * nB + bb];  i10 = gh[(size_t)a1 * nB + bb];
                      i01 = gh[(size_t)a * nB + b1];  i11 = gh[(size_t)a1 * nB + b1];
                    } else {
                      i00 = I[k][u00]; i10 = I[k][u10]; i01 = I[k][u01]; i11 = I[k][u11];
                    }
                    const double b00 = (1 - r.fa) * (1 - r.fb), b10 = r.fa * (1 - r.fb);
                    const double b01 = (1 - r.fa) * r.fb, b11 = r.fa * r.fb;
                    const double iu = b00 * i00 + b10 * i10 + b01 * i01 + b11 * i11;
                    const double su = b00 * S[u00] + b10 * S[u10] + b01 * S[u01] + b11 * S[u11];
                    const double cu = b00 * cb[u00] + b10 * cb[u10] + b01 * cb[u01] + b11 * cb[u11];
                    const double x = 0.5 * r.ds * (cb[p] + cu);
                    const Wts<double> wt = weights(x);
                    v = wt.e * iu + wt.w0 * S[p] + wt.w1 * su;
                  }
                  I[k][p] = v;
                  pn += D.w[rg[k]] * v;
                }
                if (update) {  // the Gauss-Seidel update of S_p and the group's intensities
                  const double jn = Jb[p] + (pn - P[g * N + p]);
                  const double om = 1.0 - eb[p];
                  const double dS = (om * jn + eb[p] * Bb[p] - S[p]) / (1.0 - om * Lop[p]);
                  S[p] += dS;
                  pn = 0.0;
                  for (size_t k = 0; k < rg.size(); ++k) {
                    I[k][p] += W0[(size_t)rg[k] * N + p] * dS;
                    pn += D.w[rg[k]] * I[k][p];
                  }
                }
                if (lap == laps - 1) {  // the group's contribution to J
                  Jb[p] = Jb[p] + (pn - P[g * N + p]);
                  P[g * N + p] = pn;
                }
              }
          }
          if (periodic)  // exchange: the outflow plane becomes the next lap's ghost
            for (size_t k = 0; k < rg.size(); ++k)
              for (int a = 0; a < nA; ++a)
                for (int bb = 0; bb < nB; ++bb)
                  ghost[k][(size_t)a * nB + bb] = I[k][cell(q_last, a, bb)];
        }
        if (it == n_gs - 1 && Itop) {  // I_top of the group's upward rays
          for (size_t k = 0; k < rg.size(); ++k) {
            const int r = rg[k];
            if (!rays[r].up) continue;
            int ru = 0;
            for (int r2 = 0; r2 < r; ++r2) ru += rays[r2].up;
            double* dst = Itop + ((int64_t)b * nup + ru) * plane;
            for (int64_t p = 0; p < plane; ++p) dst[p] = I[k][(int64_t)(D.n[2] - 1) * plane + p];
          }
        }
      }
    }
    const double qf = 4.0 * kPi * D.qw[b];
    for (int64_t p = 0; p < N; ++p) {
      Q[p] += qf * cb[p] * (Jb[p] - S[p]);
      if (J) J[b * N + p] = Jb[p];
      if (Sout) Sout[b * N + p] = S[p];
    }
  }
  return 0;
}

// Reverse-mode derivative of forward() for T = double.
int adjoint(const Desc& D, const double* chi, const double* S, const double* gQ,
            const double* gJ, const double* gItop, double* dS, double* dchi, int nt) {
  const int64_t N = D.cells();
  std::vector<Ray> rays(D.nr);
  for (int r = 0; r < D.nr; ++r)
    if (!make_ray(D, D.mu + 3 * r, rays[r])) return -1;
  std::vector<std::vector<double>> store;
  std::vector<double> Q(N), Jall;
  {
    // Forward with every sweep kept.
    int rc = forward<double>(D, chi, S, Q.data(), nullptr, nullptr, nt, &store, &Jall);
    if (rc) return rc;
  }
  const int64_t plane = (int64_t)D.n[0] * D.n[1];
  int nup = 0;
  for (int r = 0; r < D.nr; ++r) nup += rays[r].up;
  size_t si = 0;  // index into store
  std::vector<double> gJt(N), lam(N), lam_prev(N);
  for (int b = 0; b < D.nb; ++b) {
    const double* chib = chi + b * N;
    const double* Sb = S + b * N;
    const double* Jb = Jall.data() + b * N;
    double* dSb = dS + b * N;
    double* dcb = dchi + b * N;
    const double qf = 4.0 * kPi * D.qw[b];
    for (int64_t p = 0; p < N; ++p) {
      const double g = gQ ? gQ[p] : 0.0;
      gJt[p] = qf * chib[p] * g + (gJ ? gJ[b * N + p] : 0.0);
      dcb[p] = qf * (Jb[p] - Sb[p]) * g;
      dSb[p] = -qf * chib[p] * g;
    }
    int ru = 0;
    for (int r = 0; r < D.nr; ++r) {
      const Ray& R = rays[r];
      const int na = D.n[R.axis], nA = D.n[R.ea], nB = D.n[R.eb];
      const bool periodic = R.axis != 2;
      const int sweeps = periodic ? D.n_iter : 1;
      const size_t first_store = si;
      si += sweeps;
      auto cell = [&](int q, int a, int bb) {
        int c[3];
        c[R.axis] = q; c[R.ea] = a; c[R.eb] = bb;
        return D.at(c[0], c[1], c[2]);
      };
      auto kz = [&](int q, int a, int bb) {
        int c[3];
        c[R.axis] = q; c[R.ea] = a; c[R.eb] = bb;
        return c[2];
      };
      const double b00 = (1 - R.fa) * (1 - R.fb), b10 = R.fa * (1 - R.fb);
      const double b01 = (1 - R.fa) * R.fb, b11 = R.fa * R.fb;
      const int q_first = R.sa > 0 ? 0 : na - 1;
      const int q_last = R.sa > 0 ? na - 1 : 0;
      // seeds of the last sweep
      for (int64_t p = 0; p < N; ++p) lam[p] = D.w[r] * gJt[p];
      if (R.up) {
        if (gItop) {
          const double* g = gItop + ((int64_t)b * nup + ru) * plane;
          for (int64_t p = 0; p < plane; ++p) lam[(int64_t)(D.n[2] - 1) * plane + p] += g[p];
        }
        ++ru;
      }
      std::vector<double> lamG(periodic ? (size_t)nA * nB : 0);
      for (int sweep = sweeps - 1; sweep >= 0; --sweep) {
        const std::vector<double>& I = store[first_store + sweep];
        const std::vector<double>* Iprev = sweep > 0 ? &store[first_store + sweep - 1] : nullptr;
        std::fill(lamG.begin(), lamG.end(), 0.0);
        for (int t = na - 1; t >= (periodic ? 0 : 1); --t) {
          const int q = q_first + R.sa * t;
          const int qu = wrap(q - R.sa, na);
          const bool from_ghost = periodic && t == 0;
          for (int a = 0; a < nA; ++a)
            for (int bb = 0; bb < nB; ++bb) {
              const int64_t p = cell(q, a, bb);
              const double lp = lam[p];
              if (is_bc_layer(D, R, kz(q, a, bb))) continue;  // handled below
              if (lp == 0.0) continue;
              const int a1 = R.ea == 2 ? a - R.sea : wrap(a - R.sea, nA);
              const int b1 = R.eb == 2 ? bb - R.seb : wrap(bb - R.seb, nB);
              const int64_t u[4] = {cell(qu, a, bb), cell(qu, a1, bb), cell(qu, a, b1), cell(qu, a1, b1)};
              const double beta[4] = {b00, b10, b01, b11};
              const size_t gidx[4] = {(size_t)a * nB + bb, (size_t)a1 * nB + bb,
                                      (size_t)a * nB + b1, (size_t)a1 * nB + b1};
              double iu = 0, su = 0, cu = 0;
              for (int c = 0; c < 4; ++c) {
                double iv;
                if (from_ghost) {
                  if (Iprev) iv = (*Iprev)[u[c]];  // ghost = previous sweep's outflow plane (qu is the outflow plane)
                  else {
                    const int kc = (int)(u[c] / plane);
                    iv = is_bc_layer(D, R, kc) ? bc_value(D, R, Sb[u[c]]) : Sb[u[c]];
                  }
                } else {
                  iv = I[u[c]];
                }
                iu += beta[c] * iv;
                su += beta[c] * Sb[u[c]];
                cu += beta[c] * chib[u[c]];
              }
              const double x = 0.5 * R.ds * (chib[p] + cu);
              const Wts<double> wt = weights(x);
              const double wx = w1_over_x(x, wt.e);
              // I_p = e iu + w0 S_p + w1 su
              const double gx = lp * (-wt.e * iu + wx * Sb[p] + (wt.e - wx) * su);
              dSb[p] += wt.w0 * lp;
              dcb[p] += 0.5 * R.ds * gx;
              for (int c = 0; c < 4; ++c) {
                if (from_ghost) lamG[gidx[c]] += beta[c] * wt.e * lp;
                else lam[u[c]] += beta[c] * wt.e * lp;
                dSb[u[c]] += beta[c] * wt.w1 * lp;
                dchi[b * N + u[c]] += beta[c] * 0.5 * R.ds * gx;
              }
            }
        }
        // Boundary-layer cells of this sweep: I = S contributes to dS.
        for (int q = 0; q < na; ++q)
          for (int a = 0; a < nA; ++a)
            for (int bb = 0; bb < nB; ++bb)
              if (is_bc_layer(D, R, kz(q, a, bb))) {
                const bool thermal = R.up ? D.bot == 0 : D.top == 1;
                if (thermal) dSb[cell(q, a, bb)] += lam[cell(q, a, bb)];
              }
        if (!periodic) break;
        // Ghost sensitivities flow into the previous sweep's outflow plane, or
        // into the initial ghost (I = S of the wrapped plane).
        std::fill(lam.begin(), lam.end(), 0.0);
        for (int a = 0; a < nA; ++a)
          for (int bb = 0; bb < nB; ++bb) {
            const double g = lamG[(size_t)a * nB + bb];
            const int64_t p = cell(q_last, a, bb);
            if (sweep > 0) {
              lam[p] += g;
            } else if (is_bc_layer(D, R, kz(q_last, a, bb))) {
              const bool thermal = R.up ? D.bot == 0 : D.top == 1;
              if (thermal) dSb[p] += g;
            } else {
              dSb[p] += g;
            }
          }
      }
    }
  }
  return 0;
}

// Heating by the flux divergence, QF = -(dFx/dx + dFy/dy + dFz/dz): central
// differences, periodic in x and y; in z one-sided second-order differences in
// the bottom and top layers (first-order differences when nz = 2).
void flux_divergence(const Desc& D, const double* F, double* QF) {
  const int nx = D.n[0], ny = D.n[1], nz = D.n[2];
  const int64_t N = D.cells();
  const double* Fx = F;
  const double* Fy = F + N;
  const double* Fz = F + 2 * N;
  for (int k = 0; k < nz; ++k)
    for (int j = 0; j < ny; ++j)
      for (int i = 0; i < nx; ++i) {
        const int ip = (i + 1) % nx, im = (i + nx - 1) % nx;
        const int jp = (j + 1) % ny, jm = (j + ny - 1) % ny;
        const double ddx = (Fx[D.at(ip, j, k)] - Fx[D.at(im, j, k)]) / (2 * D.d[0]);
        const double ddy = (Fy[D.at(i, jp, k)] - Fy[D.at(i, jm, k)]) / (2 * D.d[1]);
        double ddz;
        if (nz == 2) {
          ddz = (Fz[D.at(i, j, 1)] - Fz[D.at(i, j, 0)]) / D.d[2];
        } else if (k == 0) {
          ddz = (-3 * Fz[D.at(i, j, 0)] + 4 * Fz[D.at(i, j, 1)] - Fz[D.at(i, j, 2)]) / (2 * D.d[2]);
        } else if (k == nz - 1) {
          ddz = (3 * Fz[D.at(i, j, k)] - 4 * Fz[D.at(i, j, k - 1)] + Fz[D.at(i, j, k - 2)]) /
                (2 * D.d[2]);
        } else {
          ddz = (Fz[D.at(i, j, k + 1)] - Fz[D.at(i, j, k - 1)]) / (2 * D.d[2]);
        }
        QF[D.at(i, j, k)] = -(ddx + ddy + ddz);
      }
}

// ---------------------------------------------------------------------------
// Subdomain decomposition with lagged exchange.  The paper's radiation
// transport runs on a 3D domain decomposition: each subdomain integrates its
// rays from the boundary intensities its upwind neighbours produced in the
// previous iteration, sends its own outflow intensities downstream, and the
// iteration (integrate, write buffers, exchange, error with a global maximum)
// repeats until the boundary intensities have converged.
//
// Here the grid is cut into sub[0] x sub[1] x sub[2] blocks along x, y and z
// (block b of m along an axis of n cells holds cells [b n / m, (b + 1) n / m)).
// Iteration k = 1, 2, ... of block s computes every cell of s that is not in
// a boundary layer, in the ray's sweep order.  An upwind corner u of cell p
// (in the previous plane along the dominant axis, with the periodic wrap) is
// taken from iteration k when u lies in s and p is not in the first plane of
// s along the ray (that plane's upwind plane belongs to the upstream block, or
// is the block's own outflow plane across the periodic wrap); otherwise it is
// taken from iteration k-1.  Iteration 0 is I = S off the boundary layers and
// the boundary values on them (the initial ghost plane of the undivided
// solve).  With one block this is exactly the undivided solve with n_iter
// boundary iterations.  Every ray and band iterates in lock step; with tol > 0
// the iteration stops after the first iteration k whose largest intensity
// change over all cells, rays and bands, max |I_k - I_(k-1)|, is at most tol
// times the largest |I_k| (n_iter iterations at most).

struct Blocks {
  int m[3];
  int lo(int axis, int b, const Desc& D) const { return (int)((int64_t)b * D.n[axis] / m[axis]); }
  int of(int axis, int v, const Desc& D) const {  // the block holding cell index v
    int b = (int)((int64_t)v * m[axis] / D.n[axis]);
    while (b + 1 < m[axis] && lo(axis, b + 1, D) <= v) ++b;
    while (b > 0 && lo(axis, b, D) > v) --b;
    return b;
  }
};

// One iteration of one ray over every block: Icur from Iprev.  Returns the
// largest |Icur - Iprev| and the largest |Icur| over the grid.
std::pair<double, double> block_iteration(const Desc& D, const Ray& r, const Blocks& Bk,
                                          const double* chi, const double* S,
                                          const double* Iprev, double* Icur, int nt) {
  const int na = D.n[r.axis], nA = D.n[r.ea], nB = D.n[r.eb];
  const double b00 = (1 - r.fa) * (1 - r.fb), b10 = r.fa * (1 - r.fb);
  const double b01 = (1 - r.fa) * r.fb, b11 = r.fa * r.fb;
  auto cell = [&](int q, int a, int b) {
    int c[3];
    c[r.axis] = q; c[r.ea] = a; c[r.eb] = b;
    return D.at(c[0], c[1], c[2]);
  };
  auto kz = [&](int q, int a, int b) {
    int c[3];
    c[r.axis] = q; c[r.ea] = a; c[r.eb] = b;
    return c[2];
  };
  // boundary layers: set
  for (int q = 0; q < na; ++q)
    for (int a = 0; a < nA; ++a)
      for (int b = 0; b < nB; ++b)
        if (is_bc_layer(D, r, kz(q, a, b))) {
          const int64_t p = cell(q, a, b);
          Icur[p] = bc_value(D, r, S[p]);
        }
  for (int sq = 0; sq < Bk.m[r.axis]; ++sq)
    for (int sa = 0; sa < Bk.m[r.ea]; ++sa)
      for (int sb = 0; sb < Bk.m[r.eb]; ++sb) {
        const int q0 = Bk.lo(r.axis, sq, D), q1 = Bk.lo(r.axis, sq + 1, D);
        const int a0 = Bk.lo(r.ea, sa, D), a1e = Bk.lo(r.ea, sa + 1, D);
        const int bb0 = Bk.lo(r.eb, sb, D), b1e = Bk.lo(r.eb, sb + 1, D);
        const int first = r.sa > 0 ? q0 : q1 - 1;
        for (int t = 0; t < q1 - q0; ++t) {
          const int q = first + r.sa * t;
          const int qu = wrap(q - r.sa, na);
          const bool first_plane = t == 0;
#pragma omp parallel for collapse(2) num_threads(nt) schedule(static)
          for (int a = a0; a < a1e; ++a)
            for (int b = bb0; b < b1e; ++b) {
              if (is_bc_layer(D, r, kz(q, a, b))) continue;
              const int64_t p = cell(q, a, b);
              const int a1 = r.ea == 2 ? a - r.sea : wrap(a - r.sea, nA);
              const int b1 = r.eb == 2 ? b - r.seb : wrap(b - r.seb, nB);
              const int64_t u00 = cell(qu, a, b), u10 = cell(qu, a1, b);
              const int64_t u01 = cell(qu, a, b1), u11 = cell(qu, a1, b1);
              // current iteration only for corners of this block behind its first plane
              const bool in_a = a1 >= a0 && a1 < a1e, in_b = b1 >= bb0 && b1 < b1e;
              const double* s00 = first_plane ? Iprev : Icur;
              const double* s10 = first_plane || !in_a ? Iprev : Icur;
              const double* s01 = first_plane || !in_b ? Iprev : Icur;
              const double* s11 = first_plane || !in_a || !in_b ? Iprev : Icur;
              const double i00 = s00[u00], i10 = s10[u10], i01 = s01[u01], i11 = s11[u11];
              const double iu = b00 * i00 + b10 * i10 + b01 * i01 + b11 * i11;
              const double su = b00 * S[u00] + b10 * S[u10] + b01 * S[u01] + b11 * S[u11];
              const double cu = b00 * chi[u00] + b10 * chi[u10] + b01 * chi[u01] + b11 * chi[u11];
              const double x = 0.5 * r.ds * (chi[p] + cu);
              const Wts<double> wt = weights(x);
              Icur[p] = wt.e * iu + wt.w0 * S[p] + wt.w1 * su;
            }
        }
      }
  double diff = 0.0, scale = 0.0;
  for (int64_t p = 0; p < D.cells(); ++p) {
    diff = std::max(diff, std::fabs(Icur[p] - Iprev[p]));
    scale = std::max(scale, std::fabs(Icur[p]));
  }
  return {diff, scale};
}

// The decomposed solve of every band and ray; Q, J, Itop as in forward().
// Iall (optional) receives the final intensities [nb][nr][N]; the return
// value is the number of iterations run (or -1).
int forward_blocks(const Desc& D, const Blocks& Bk, const double* chi, const double* S,
                   double* Q, double* J, double* Itop, double* Iall, int nt) {
  const int64_t N = D.cells();
  std::vector<Ray> rays(D.nr);
  for (int r = 0; r < D.nr; ++r)
    if (!make_ray(D, D.mu + 3 * r, rays[r])) return -1;
  const size_t nf = (size_t)D.nb * D.nr;
  std::vector<std::vector<double>> prev(nf, std::vector<double>(N)), cur(nf, std::vector<double>(N));
  // iteration 0: I = S, boundary layers at their values
  for (int b = 0; b < D.nb; ++b)
    for (int r = 0; r < D.nr; ++r) {
      std::vector<double>& I0 = prev[(size_t)b * D.nr + r];
      for (int k = 0; k < D.n[2]; ++k)
        for (int64_t p = (int64_t)k * D.n[0] * D.n[1]; p < (int64_t)(k + 1) * D.n[0] * D.n[1]; ++p)
          I0[p] = is_bc_layer(D, rays[r], k) ? bc_value(D, rays[r], S[b * N + p]) : S[b * N + p];
    }
  int used = 0;
  for (int it = 0; it < D.n_iter; ++it) {
    double diff = 0.0, scale = 0.0;
    for (int b = 0; b < D.nb; ++b)
      for (int r = 0; r < D.nr; ++r) {
        const size_t f = (size_t)b * D.nr + r;
        const auto ds = block_iteration(D, rays[r], Bk, chi + b * N, S + b * N, prev[f].data(),
                                        cur[f].data(), nt);
        diff = std::max(diff, ds.first);
        scale = std::max(scale, ds.second);
      }
    std::swap(prev, cur);  // prev holds iteration it + 1
    used = it + 1;
    if (D.tol > 0 && diff <= D.tol * scale) break;
  }
  // flux step from the last iteration run
  const int64_t plane = (int64_t)D.n[0] * D.n[1];
  int nup = 0;
  for (int r = 0; r < D.nr; ++r) nup += rays[r].up;
  for (int64_t p = 0; p < N; ++p) Q[p] = 0.0;
  std::vector<double> Jb(N);
  for (int b = 0; b < D.nb; ++b) {
    for (int64_t p = 0; p < N; ++p) Jb[p] = 0.0;
    int ru = 0;
    for (int r = 0; r < D.nr; ++r) {
      const std::vector<double>& I = prev[(size_t)b * D.nr + r];
      for (int64_t p = 0; p < N; ++p) Jb[p] += D.w[r] * I[p];
      if (Iall) std::copy(I.begin(), I.end(), Iall + ((size_t)b * D.nr + r) * N);
      if (rays[r].up) {
        if (Itop) {
          double* dst = Itop + ((int64_t)b * nup + ru) * plane;
          for (int64_t p = 0; p < plane; ++p) dst[p] = I[(int64_t)(D.n[2] - 1) * plane + p];
        }
        ++ru;
      }
    }
    const double qf = 4.0 * kPi * D.qw[b];
    for (int64_t p = 0; p < N; ++p) Q[p] += qf * chi[b * N + p] * (Jb[p] - S[b * N + p]);
    if (J) std::memcpy(J + b * N, Jb.data(), sizeof(double) * N);
  }
  return used;
}

Desc make_desc(int nx, int ny, int nz, double dx, double dy, double dz, int nb, int nr,
               const double* mu, const double* w, const double* qw, int bot, int top,
               double ibot, int n_iter) {
  Desc D;
  D.n[0] = nx; D.n[1] = ny; D.n[2] = nz;
  D.d[0] = dx; D.d[1] = dy; D.d[2] = dz;
  D.nb = nb; D.nr = nr; D.mu = mu; D.w = w; D.qw = qw;
  D.bot = bot; D.top = top; D.ibot = ibot; D.n_iter = n_iter;
  return D;
}

bool valid(const Desc& D) {
  for (int d = 0; d < 3; ++d)
    if (D.n[d] < 2 || !(D.d[d] > 0)) return false;
  return D.nb >= 1 && D.nr >= 1 && D.n_iter >= 1;
}

}  // namespace

extern "C" {

// Forward solve from extinction chi [nb][N] and source S [nb][N] (C order
// [z][y][x]).  Q [N] is written; J [nb][N] and Itop [nb][n_up][ny][nx] if not
// null.  Returns 0, or -1 on invalid input.
int oracle_solve_chi(int nx, int ny, int nz, double dx, double dy, double dz, int nb, int nr,
                     const double* mu, const double* w, const double* qw, int bot, int top,
                     double ibot, int n_iter, const double* chi, const double* S, double* Q,
                     double* J, double* Itop, int nthreads) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, nb, nr, mu, w, qw, bot, top, ibot, n_iter);
  if (!valid(D)) return -1;
  return forward<double>(D, chi, S, Q, J, Itop, nthreads > 0 ? nthreads : 1, nullptr, nullptr);
}

// Same, from kappa [nb][N] and rho [N]: chi_b = kappa_b * rho.
int oracle_solve(int nx, int ny, int nz, double dx, double dy, double dz, int nb, int nr,
                 const double* mu, const double* w, const double* qw, int bot, int top,
                 double ibot, int n_iter, const double* kappa, const double* rho,
                 const double* S, double* Q, double* J, double* Itop, int nthreads) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, nb, nr, mu, w, qw, bot, top, ibot, n_iter);
  if (!valid(D)) return -1;
  const int64_t N = D.cells();
  std::vector<double> chi((size_t)nb * N);
  for (int b = 0; b < nb; ++b)
    for (int64_t p = 0; p < N; ++p) chi[b * N + p] = kappa[b * N + p] * rho[p];
  return forward<double>(D, chi.data(), S, Q, J, Itop, nthreads > 0 ? nthreads : 1, nullptr,
                         nullptr);
}

// Gauss-Seidel scattering (forward_gs): kappa, rho as oracle_solve, B the
// thermal source [nb][N] and eps [nb][N] the photon destruction probability;
// n_gs iterations; Q, J, Itop as oracle_solve and Sout [nb][N] the final
// source function (J, Itop, Sout may be null).
int oracle_solve_gs(int nx, int ny, int nz, double dx, double dy, double dz, int nb, int nr,
                    const double* mu, const double* w, const double* qw, int bot, int top,
                    double ibot, int n_iter, const double* kappa, const double* rho,
                    const double* B, const double* eps, int n_gs, double* Q, double* J,
                    double* Itop, double* Sout) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, nb, nr, mu, w, qw, bot, top, ibot, n_iter);
  if (!valid(D) || n_gs < 1) return -1;
  const int64_t N = D.cells();
  std::vector<double> chi((size_t)nb * N);
  for (int b = 0; b < nb; ++b)
    for (int64_t p = 0; p < N; ++p) chi[b * N + p] = kappa[b * N + p] * rho[p];
  return forward_gs(D, chi.data(), B, eps, n_gs, Q, J, Itop, Sout);
}

// The D-form second mode (forward_dform): inputs and outputs as oracle_solve.
int oracle_solve_dform(int nx, int ny, int nz, double dx, double dy, double dz, int nb, int nr,
                       const double* mu, const double* w, const double* qw, int bot, int top,
                       double ibot, int n_iter, const double* kappa, const double* rho,
                       const double* S, double* Q, double* J, double* Itop) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, nb, nr, mu, w, qw, bot, top, ibot, n_iter);
  if (!valid(D)) return -1;
  const int64_t N = D.cells();
  std::vector<double> chi((size_t)nb * N);
  for (int b = 0; b < nb; ++b)
    for (int64_t p = 0; p < N; ++p) chi[b * N + p] = kappa[b * N + p] * rho[p];
  return forward_dform(D, chi.data(), S, Q, J, Itop);
}

// Forward solve with the radiative flux vector F [3][N] (x, y, z components,
// summed over bands with qweight) and, if QF is not null, the heating -div F
// [N]; Q, J and Itop as in oracle_solve (J, Itop may be null).
int oracle_flux(int nx, int ny, int nz, double dx, double dy, double dz, int nb, int nr,
                const double* mu, const double* w, const double* qw, int bot, int top,
                double ibot, int n_iter, const double* kappa, const double* rho,
                const double* S, double* Q, double* J, double* Itop, double* F, double* QF,
                int nthreads) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, nb, nr, mu, w, qw, bot, top, ibot, n_iter);
  if (!valid(D) || !F) return -1;
  const int64_t N = D.cells();
  std::vector<double> chi((size_t)nb * N);
  for (int b = 0; b < nb; ++b)
    for (int64_t p = 0; p < N; ++p) chi[b * N + p] = kappa[b * N + p] * rho[p];
  const int rc = forward<double>(D, chi.data(), S, Q, J, Itop, nthreads > 0 ? nthreads : 1,
                                 nullptr, nullptr, F);
  if (rc) return rc;
  if (QF) flux_divergence(D, F, QF);
  return 0;
}

// Forward solve with tolerance-driven boundary iteration (tol > 0; n_iter is
// the largest sweep count): Q, J, Itop as in oracle_solve, F and QF as in
// oracle_flux when F is not null, and sweeps [nb][nr] the sweeps each ray
// used.
int oracle_solve_tol(int nx, int ny, int nz, double dx, double dy, double dz, int nb, int nr,
                     const double* mu, const double* w, const double* qw, int bot, int top,
                     double ibot, int n_iter, double tol, const double* kappa, const double* rho,
                     const double* S, double* Q, double* J, double* Itop, double* F, double* QF,
                     int* sweeps, int nthreads) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, nb, nr, mu, w, qw, bot, top, ibot, n_iter);
  if (!valid(D) || !(tol > 0) || !std::isfinite(tol)) return -1;
  D.tol = tol;
  const int64_t N = D.cells();
  std::vector<double> chi((size_t)nb * N);
  for (int b = 0; b < nb; ++b)
    for (int64_t p = 0; p < N; ++p) chi[b * N + p] = kappa[b * N + p] * rho[p];
  const int rc = forward<double>(D, chi.data(), S, Q, J, Itop, nthreads > 0 ? nthreads : 1,
                                 nullptr, nullptr, F, sweeps);
  if (rc) return rc;
  if (F && QF) flux_divergence(D, F, QF);
  return 0;
}

// Warm start: the solve (with tol > 0 tolerance-driven, else n_iter sweeps)
// from the given initial ghost planes gin (or null: I = S), writing the final
// ghost planes to gout (if not null), both [nb][nr][nz][max(nx, ny)] (entries
// of z-dominant rays untouched); Q, J, Itop as oracle_solve; sweeps [nb][nr]
// (tol > 0 only, may be null).
int oracle_solve_warm(int nx, int ny, int nz, double dx, double dy, double dz, int nb, int nr,
                      const double* mu, const double* w, const double* qw, int bot, int top,
                      double ibot, int n_iter, double tol, const double* kappa, const double* rho,
                      const double* S, const double* gin, double* gout, double* Q, double* J,
                      double* Itop, int* sweeps, int nthreads) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, nb, nr, mu, w, qw, bot, top, ibot, n_iter);
  if (!valid(D) || !(tol >= 0) || !std::isfinite(tol)) return -1;
  D.tol = tol;
  D.gin = gin;
  D.gout = gout;
  const int64_t N = D.cells();
  std::vector<double> chi((size_t)nb * N);
  for (int b = 0; b < nb; ++b)
    for (int64_t p = 0; p < N; ++p) chi[b * N + p] = kappa[b * N + p] * rho[p];
  return forward<double>(D, chi.data(), S, Q, J, Itop, nthreads > 0 ? nthreads : 1, nullptr,
                         nullptr, nullptr, sweeps);
}

// Divergence heating -div F [N] of a given flux field F [3][N] (the same
// differences as oracle_flux).
int oracle_flux_divergence(int nx, int ny, int nz, double dx, double dy, double dz,
                           const double* F, double* QF) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, 1, 1, nullptr, nullptr, nullptr, 0, 0, 0.0, 1);
  for (int d = 0; d < 3; ++d)
    if (D.n[d] < 2 || !(D.d[d] > 0)) return -1;
  flux_divergence(D, F, QF);
  return 0;
}

// Intensity of one ray for one band (I [N]) after all its sweeps.
int oracle_ray(int nx, int ny, int nz, double dx, double dy, double dz, const double* mu3,
               int bot, int top, double ibot, int n_iter, const double* chi, const double* S,
               double* I) {
  const double w1 = 1.0, q1 = 1.0;
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, 1, 1, mu3, &w1, &q1, bot, top, ibot, n_iter);
  if (!valid(D)) return -1;
  Ray r;
  if (!make_ray(D, mu3, r)) return -1;
  solve_ray<double>(D, r, chi, S, I, nullptr, 1);
  return 0;
}

// Forward solve on sub[0] x sub[1] x sub[2] subdomains with lagged exchange
// between iterations (n_iter iterations, or tol > 0: until the largest
// intensity change is at most tol of the largest intensity).  Q, J, Itop as in
// oracle_solve (J, Itop may be null); Iall [nb][nr][N] receives the final
// intensity of every ray if not null; *iters the iterations run.
int oracle_solve_sub(int nx, int ny, int nz, double dx, double dy, double dz, int nb, int nr,
                     const double* mu, const double* w, const double* qw, int bot, int top,
                     double ibot, int n_iter, const int* sub, double tol, const double* kappa,
                     const double* rho, const double* S, double* Q, double* J, double* Itop,
                     double* Iall, int* iters, int nthreads) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, nb, nr, mu, w, qw, bot, top, ibot, n_iter);
  if (!valid(D) || !(tol >= 0) || !std::isfinite(tol)) return -1;
  Blocks Bk;
  for (int a = 0; a < 3; ++a) {
    if (sub[a] < 1 || sub[a] > D.n[a]) return -1;
    Bk.m[a] = sub[a];
  }
  D.tol = tol;
  const int64_t N = D.cells();
  std::vector<double> chi((size_t)nb * N);
  for (int b = 0; b < nb; ++b)
    for (int64_t p = 0; p < N; ++p) chi[b * N + p] = kappa[b * N + p] * rho[p];
  const int used = forward_blocks(D, Bk, chi.data(), S, Q, J, Itop, Iall,
                                  nthreads > 0 ? nthreads : 1);
  if (used < 0) return -1;
  if (iters) *iters = used;
  return 0;
}

// Linear-source weights, exposed for the weight-function pins.
void oracle_weights(double x, double* e, double* w0, double* w1, double* w1x) {
  Wts<double> wt = weights(x);
  *e = wt.e; *w0 = wt.w0; *w1 = wt.w1;
  *w1x = w1_over_x(x, wt.e);
}

// Reverse-mode gradients of L = sum(gQ Q) + sum(gJ J) + sum(gItop Itop) with
// respect to S [nb][N] and chi [nb][N].  gQ, gJ, gItop may be null.
int oracle_adjoint(int nx, int ny, int nz, double dx, double dy, double dz, int nb, int nr,
                   const double* mu, const double* w, const double* qw, int bot, int top,
                   double ibot, int n_iter, const double* chi, const double* S,
                   const double* gQ, const double* gJ, const double* gItop, double* dS,
                   double* dchi, int nthreads) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, nb, nr, mu, w, qw, bot, top, ibot, n_iter);
  if (!valid(D)) return -1;
  return adjoint(D, chi, S, gQ, gJ, gItop, dS, dchi, nthreads > 0 ? nthreads : 1);
}

// Complex-step directional derivative: chi or S (which = 1 or 0) at flat index
// `idx` of the [nb][N] array is perturbed by i*h; the imaginary parts of Q, J
// and Itop divided by h are returned (J, Itop may be null).
int oracle_complex_step(int nx, int ny, int nz, double dx, double dy, double dz, int nb,
                        int nr, const double* mu, const double* w, const double* qw, int bot,
                        int top, double ibot, int n_iter, const double* chi, const double* S,
                        int which, int64_t idx, double h, double* dQ, double* dJ,
                        double* dItop, int nthreads) {
  Desc D = make_desc(nx, ny, nz, dx, dy, dz, nb, nr, mu, w, qw, bot, top, ibot, n_iter);
  if (!valid(D)) return -1;
  const int64_t N = D.cells();
  std::vector<cplx> c(chi, chi + nb * N), s(S, S + nb * N), Q(N), J((size_t)nb * N);
  int nup = 0;
  for (int r = 0; r < nr; ++r) nup += mu[3 * r + 2] > 0;
  const int64_t plane = (int64_t)nx * ny;
  std::vector<cplx> It((size_t)nb * nup * plane);
  if (which) c[idx] += cplx(0.0, h);
  else s[idx] += cplx(0.0, h);
  int rc = forward<cplx>(D, c.data(), s.data(), Q.data(), J.data(), It.data(),
                         nthreads > 0 ? nthreads : 1, nullptr, nullptr);
  if (rc) return rc;
  for (int64_t p = 0; p < N; ++p) dQ[p] = Q[p].imag() / h;
  if (dJ)
    for (int64_t p = 0; p < nb * N; ++p) dJ[p] = J[p].imag() / h;
  if (dItop)
    for (size_t p = 0; p < It.size(); ++p) dItop[p] = It[p].imag() / h;
  return 0;
}

}  // extern "C"
