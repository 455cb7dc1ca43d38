// Kernels around the sweeps: chi preparation with the transposed copies, the
// fill kernel, the FP64 reductions of J, Q and the flux vector, the flux
// divergence, the adjoint's seeds and its gradient reduction, with their
// launch wrappers.
#include "rts_device.hpp"

namespace rts {

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


// Sets *flag when any of the n values is a NaN or an infinity (all exponent
// bits set).  Reads the values once, coalesced; a finding is one atomic OR.
template <class Real>
__global__ __launch_bounds__(256) void rts_scan_nonfinite(const Real* __restrict__ v, int64_t n,
                                                          int* flag) {
  bool bad = false;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    if constexpr (sizeof(Real) == 4) {
      const uint32_t u = __float_as_uint((float)v[i]);
      bad |= (u & 0x7f800000u) == 0x7f800000u;
    } else {
      const uint64_t u = (uint64_t)__double_as_longlong((double)v[i]);
      bad |= (u & 0x7ff0000000000000ull) == 0x7ff0000000000000ull;
    }
  }
  if (bad) atomicOr(flag, 1);
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


// ---------------------------------------------------------------------------
// launch wrappers used by the host planner

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


template <class Real>
hipError_t launch_scan_nonfinite(const void* v, int64_t n, int* flag, int cus, hipStream_t st) {
  int64_t blocks = (n + 255) / 256;
  blocks = blocks > 8 * (int64_t)cus ? 8 * (int64_t)cus : blocks;  // grid-stride beyond that
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(rts_scan_nonfinite<Real>, dim3((unsigned)blocks), dim3(256), 0, st,
                     (const Real*)v, n, flag);
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
template hipError_t launch_scan_nonfinite<float>(const void*, int64_t, int*, int, hipStream_t);
template hipError_t launch_scan_nonfinite<double>(const void*, int64_t, int*, int, hipStream_t);
template hipError_t launch_reduce<float>(const char*, const Task*, const BoxGeo&, const BoxPtrs&,
                                         hipStream_t);
template hipError_t launch_reduce<double>(const char*, const Task*, const BoxGeo&, const BoxPtrs&,
                                          hipStream_t);

template hipError_t launch_adj_seed<float>(const void*, const void*, const double*, const void*,
                                           void*, void*, double, int, int, int, hipStream_t);
template hipError_t launch_adj_seed<double>(const void*, const void*, const double*, const void*,
                                            void*, void*, double, int, int, int, hipStream_t);
template hipError_t launch_adj_reduce<float>(const char*, const Task*, const AdjTask*, const BoxGeo&,
                                             const double*, const void*, const void*, const void*,
                                             void*, void*, hipStream_t);
template hipError_t launch_adj_reduce<double>(const char*, const Task*, const AdjTask*, const BoxGeo&,
                                              const double*, const void*, const void*, const void*,
                                              void*, void*, hipStream_t);

}  // namespace rts
