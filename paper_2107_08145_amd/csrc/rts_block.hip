// Subdomain decomposition with lagged exchange on one GPU: the paper's
// domain-decomposed radiation transport (section "Summary of the Radiation
// Transport Solver": subdomains integrate with boundary intensities from their
// upwind neighbours and iterate them; the RTS core-loop figure: integrate,
// write buffers, exchange, error with a global maximum, repeat).
//
// The box is cut into blocks (subdomains).  One iteration is one launch of
// rts_block_sweep: a workgroup per (sweep task, block) sweeps the block's
// planes in the task's direction, D = I - S of its four ray slots for every
// cell of a plane, and writes them into this iteration's D field.  An upwind
// corner is read from this iteration's field when it lies in the same block
// and the cell is not in the block's first plane along the ray; otherwise
// from the previous iteration's field (the lagged boundary intensities that a
// multi-GPU run would have received from its upwind neighbours).  The fields
// of the two iteration parities alternate, so no workgroup ever waits for
// another: the launch boundary is the exchange.  Inside a workgroup a plane's
// cells are independent; the previous plane of the block is read back from
// the field after a workgroup barrier.
//
// With a tolerance, every workgroup folds the largest |D_k - D_(k-1)| and
// |I_k| of its cells into the iteration's two words (device-scope atomic max
// of non-negative doubles, which order like their bits); the next launch reads
// them first and, once the change is within tol of the largest intensity, all
// its workgroups return at once (outputs are written every iteration in that
// mode, so the last iteration run keeps them).
#include "rts_device.hpp"

namespace rts {

namespace {

// Block range [lo, hi) of block b of m along an axis of n cells.
__device__ inline int blk_lo(int n, int m, int b) { return (int)((int64_t)b * n / m); }

}  // namespace

// Iteration 0 of every task's D field: D = 0 (I = S) off the boundary
// layers, the boundary value on them.  grid.y = task, grid.x over cells.
template <class Real>
__global__ __launch_bounds__(256) void rts_block_init(BlockArgs A) {
  const Task& T = A.tasks[blockIdx.y];
  const int64_t N = T.n_cells;
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= N) return;
  // (plane, row) of view offset o = q ps + i rs + c: the larger stride is the outer index
  const int64_t ps = T.plane_stride, rs = T.row_stride;
  const int q = (int)(ps > rs ? o / ps : (o % rs) / ps);
  const int i = (int)(ps > rs ? (o % ps) / rs : o / rs);
  const Real* Sv = T.transposed ? reinterpret_cast<const Real*>(A.ws) + T.s_off
                                : reinterpret_cast<const Real*>(A.box[T.box].S) + T.s_off;
  const Real s = Sv[o];
  Real* D0 = reinterpret_cast<Real*>(A.ws) + T.dfield_off;  // parity 0
  const int q_bc = T.sa > 0 ? 0 : T.n_planes - 1;
  for (int r = 0; r < kMaxRaysPerTask; ++r) {
    const bool up = (r & 1) == 0;
    Real v = Real(0);
    if (T.z_planes) {
      if (q == q_bc) v = (Real)T.pl_a * s + (Real)T.pl_b;
    } else if (up && i == 0) {
      v = (Real)T.bu_a * s + (Real)T.bu_b;
    } else if (!up && i == T.n_rows - 1) {
      v = (Real)T.bd_a * s + (Real)T.bd_b;
    }
    D0[(int64_t)r * N + o] = v;
  }
}

// One iteration: grid.x = block (blocks of the task's box beyond its count
// return), grid.y = task.
template <class Real>
__global__ __launch_bounds__(1024) void rts_block_sweep(BlockArgs A) {
  constexpr int R = kMaxRaysPerTask;
  const Task& T = A.tasks[blockIdx.y];
  const int nbc = T.nblk[0], nbr = T.nblk[1], nbp = T.nblk[2];
  if ((int)blockIdx.x >= nbc * nbr * nbp || A.iter >= T.iters) return;
  const int64_t N = T.n_cells;
  uint64_t* tw = T.btol_off >= 0 ? reinterpret_cast<uint64_t*>(A.ws) + T.btol_off : nullptr;
  // outputs from the last iteration (every iteration with a tolerance: the last one run)
  const bool outputs = tw != nullptr || A.iter == T.iters - 1;
  if (tw && A.iter > 0) {
    // the previous iteration's maxima decide (every workgroup reads the same words)
    const double dd = __longlong_as_double((long long)tw[2 * (A.iter - 1)]);
    const double dm = __longlong_as_double((long long)tw[2 * (A.iter - 1) + 1]);
    if (dd <= T.tol * dm) return;
  }
  const int bc = (int)blockIdx.x % nbc;
  const int br = ((int)blockIdx.x / nbc) % nbr;
  const int bp = (int)blockIdx.x / (nbc * nbr);
  const int W = T.n_cols, nr = T.n_rows, na = T.n_planes;
  const int c0 = blk_lo(W, nbc, bc), c1 = blk_lo(W, nbc, bc + 1);
  const int r0 = blk_lo(nr, nbr, br), r1 = blk_lo(nr, nbr, br + 1);
  const int p0 = blk_lo(na, nbp, bp), p1 = blk_lo(na, nbp, bp + 1);
  const int ncb = c1 - c0, ncell = ncb * (r1 - r0);
  const int ps = (int)T.plane_stride, rs = (int)T.row_stride;
  const bool per = T.row_periodic != 0;
  const Real* chi = reinterpret_cast<const Real*>(A.ws) + T.chi_off;
  const Real* Sv = T.transposed ? reinterpret_cast<const Real*>(A.ws) + T.s_off
                                : reinterpret_cast<const Real*>(A.box[T.box].S) + T.s_off;
  // launch A.iter computes iteration A.iter + 1 from iteration A.iter (iteration
  // 0 is rts_block_init's field, parity 0)
  Real* Dcur = reinterpret_cast<Real*>(A.ws) + T.dfield_off + (int64_t)((A.iter + 1) & 1) * R * N;
  const Real* Dprv = reinterpret_cast<const Real*>(A.ws) + T.dfield_off +
                     (int64_t)(A.iter & 1) * R * N;
  Real* P = reinterpret_cast<Real*>(A.ws) + T.part_off;
  Real* Itop = reinterpret_cast<Real*>(A.box[T.box].I_top);
  // per-slot constants; FP32 folds log2(e) into ds/2 (rts_exp_step)
  const Real kx = sizeof(Real) == 4 ? Real(1.4426950408889634) : Real(1);
  Real f1[R], f2[R], hds[R], wgt[R];
  for (int r = 0; r < R; ++r) {
    f1[r] = (Real)T.ray[r].f1;
    f2[r] = (Real)T.ray[r].f2;
    hds[r] = (Real)T.ray[r].hds * kx;
    wgt[r] = (Real)T.ray[r].w;
  }
  const int q_bc = T.sa > 0 ? 0 : na - 1;
  const int first = T.sa > 0 ? p0 : p1 - 1;
  double dmax = 0.0, imax = 0.0;
  for (int t = 0; t < p1 - p0; ++t) {
    const int q = first + T.sa * t;
    const int qu = q - T.sa < 0 ? q - T.sa + na : (q - T.sa >= na ? q - T.sa - na : q - T.sa);
    const bool first_plane = t == 0;
    for (int idx = threadIdx.x; idx < ncell; idx += blockDim.x) {
      const int i = r0 + idx / ncb, c = c0 + idx % ncb;
      const int64_t o = (int64_t)q * ps + (int64_t)i * rs + c;
      const Real sp = Sv[o], cp = chi[o];
      Real Dn[R];
      for (int r = 0; r < R; ++r) {
        const bool up = (r & 1) == 0;
        if (T.ray[r].ray < 0) {  // unused slot
          Dn[r] = Real(0);
          continue;
        }
        if (T.z_planes ? q == q_bc : (up ? i == 0 : i == nr - 1)) {
          // boundary layer: set, not integrated
          Dn[r] = T.z_planes ? (Real)T.pl_a * sp + (Real)T.pl_b
                             : (up ? (Real)T.bu_a * sp + (Real)T.bu_b : (Real)T.bd_a * sp + (Real)T.bd_b);
          continue;
        }
        // upwind corners: column c - 1 (slots 0, 1) or c + 1, row i - 1 (even
        // slots) or i + 1, periodic in columns (and rows when they wrap)
        int cu = r < 2 ? c - 1 : c + 1;
        cu = cu < 0 ? cu + W : (cu >= W ? cu - W : cu);
        int iu = up ? i - 1 : i + 1;
        if (per) iu = iu < 0 ? iu + nr : (iu >= nr ? iu - nr : iu);
        const bool in_c = cu >= c0 && cu < c1, in_r = iu >= r0 && iu < r1;
        const int64_t b = (int64_t)qu * ps;
        const int64_t u00 = b + (int64_t)i * rs + c, u10 = b + (int64_t)i * rs + cu;
        const int64_t u01 = b + (int64_t)iu * rs + c, u11 = b + (int64_t)iu * rs + cu;
        const Real* f = Dcur + (int64_t)r * N;
        const Real* g = Dprv + (int64_t)r * N;
        const Real d00 = (first_plane ? g : f)[u00];
        const Real d10 = (first_plane || !in_c ? g : f)[u10];
        const Real d01 = (first_plane || !in_r ? g : f)[u01];
        const Real d11 = (first_plane || !in_c || !in_r ? g : f)[u11];
        // bilinear in the upwind face: along columns (f1), then rows (f2)
        const Real bd = lerp(lerp(d00, d10, f1[r]), lerp(d01, d11, f1[r]), f2[r]);
        const Real bs = lerp(lerp(Sv[u00], Sv[u10], f1[r]), lerp(Sv[u01], Sv[u11], f1[r]), f2[r]);
        const Real bx = lerp(lerp(chi[u00], chi[u10], f1[r]), lerp(chi[u01], chi[u11], f1[r]), f2[r]);
        const Real xs = hds[r] * (cp + bx);
        const Real e = rts_exp_step(xs);
        const Real cw = rts_small_step(xs) ? rts_c_series(xs) : rts_c_closed(xs, e);
        Dn[r] = fmad(e, bd, cw * (bs - sp));
      }
      for (int r = 0; r < R; ++r) {
        if (tw && T.ray[r].ray >= 0) {
          dmax = fmax(dmax, (double)fabs(Dn[r] - Dprv[(int64_t)r * N + o]));
          imax = fmax(imax, (double)fabs(Dn[r] + sp));
        }
        Dcur[(int64_t)r * N + o] = Dn[r];
      }
      if (outputs) {
        P[o] = fmad(wgt[1], Dn[1], wgt[0] * Dn[0]) + fmad(wgt[3], Dn[3], wgt[2] * Dn[2]);
        if (Itop && (T.z_planes ? q == T.it_top : i == T.it_top)) {
          for (int r = 0; r < R; ++r) {
            const int it = T.ray[r].itop;
            if (it >= 0)
              Itop[T.it_off + it * T.it_ray + (int64_t)q * T.itp + (int64_t)i * T.itr +
                   (int64_t)c * T.itc] = sp + Dn[r];
          }
        }
      }
    }
    __syncthreads();  // this plane of the field is complete for the next one
  }
  if (tw) {
    __shared__ double red[2][16];
    for (int off = 32; off >= 1; off >>= 1) {
      dmax = fmax(dmax, __shfl_xor(dmax, off));
      imax = fmax(imax, __shfl_xor(imax, off));
    }
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = dmax;
      red[1][threadIdx.x >> 6] = imax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < (int)(blockDim.x + 63) / 64; ++w) {
        dmax = fmax(dmax, red[0][w]);
        imax = fmax(imax, red[1][w]);
      }
      atomicMax(reinterpret_cast<unsigned long long*>(&tw[2 * A.iter]),
                (unsigned long long)__double_as_longlong(dmax));
      atomicMax(reinterpret_cast<unsigned long long*>(&tw[2 * A.iter + 1]),
                (unsigned long long)__double_as_longlong(imax));
    }
  }
}

template <class Real>
hipError_t launch_block_init(const BlockArgs& a, int64_t max_cells, hipStream_t st) {
  const dim3 grid((unsigned)((max_cells + 255) / 256), (unsigned)a.ntasks);
  rts_block_init<Real><<<grid, dim3(256), 0, st>>>(a);
  return hipGetLastError();
}

template <class Real>
hipError_t launch_block_sweep(const BlockArgs& a, int max_blocks, int threads, hipStream_t st) {
  if (threads < 64 || threads > 1024 || threads % 64) return hipErrorInvalidValue;
  const dim3 grid((unsigned)max_blocks, (unsigned)a.ntasks);
  rts_block_sweep<Real><<<grid, dim3((unsigned)threads), 0, st>>>(a);
  return hipGetLastError();
}

template hipError_t launch_block_init<float>(const BlockArgs&, int64_t, hipStream_t);
template hipError_t launch_block_init<double>(const BlockArgs&, int64_t, hipStream_t);
template hipError_t launch_block_sweep<float>(const BlockArgs&, int, int, hipStream_t);
template hipError_t launch_block_sweep<double>(const BlockArgs&, int, int, hipStream_t);

}  // namespace rts
