// Internal structures shared by the host planner (rts_host.cpp) and the gfx950
// kernels (rts_device.hpp, rts_sweep.hpp, rts_reverse.hpp, rts_misc.hip).  Not
// part of the public ABI.
#pragma once
#include <stdint.h>

namespace rts {

constexpr int kMaxRaysPerTask = 4;
constexpr int kMaxBoxes = 16;
constexpr int kMaxCols = 1024;  // one thread per column of the sweep plane

// One ray slot inside a sweep task.  "cols" is the contiguous in-plane axis
// (always periodic), "rows" the other in-plane axis.  Slot k's upwind column
// is c-1 for k < 2 (else c+1) and its upwind row i-1 for even k (else i+1);
// an unused slot has w = 0, f1 = f2 = 0, ds = 0, itop = -1.
struct TaskRay {
  double f1, f2;   // upwind fractions along cols and rows
  double hds;      // ds / 2
  double w;        // quadrature weight
  int32_t itop;    // index among rays with mu_z > 0, or -1
  int32_t ray;     // input ray index, or -1 for an unused slot
  double wm[3];    // w mu along (cols, rows, plane axis): weights of the flux partials
};

// One sweep task: up to four rays of one band of one box that share the
// dominant axis and its direction.  The task is split into strips of rows;
// each strip is processed by one workgroup that marches through the planes.
struct Task {
  int32_t box, band;
  int32_t n_planes, n_rows, n_cols;
  int32_t sa;              // +1 / -1 along the plane axis
  int32_t laps;            // sweeps over the plane axis (1 when planes are z)
  int32_t z_planes;        // planes are z: the first plane is the boundary layer
  int32_t row_periodic;    // rows wrap (planes are z) or end at boundaries (rows are z)
  int32_t nrays;
  int32_t rows_per_strip, strips;
  int32_t ticket0;         // first queue ticket of this task
  int32_t transposed;      // chi/S read from the [x][z][y] copies
  int32_t it_top;          // plane (z_planes) or row (otherwise) of the top layer
  int32_t uni;             // all four slots share f1, f2, ds and w
  int64_t plane_stride, row_stride;  // element strides of the view (col stride 1)
  int64_t chi_off;         // element offset of this band's chi view in the workspace
  int64_t s_off;           // element offset of S: into the box's S (natural) or workspace
  int64_t part_off;        // element offset of the partial sum array in the workspace
  int64_t flux_off;        // element offset of the flux partials along (cols, rows[, plane
                           // axis]) [2 or 3][n_cells], or -1; with uni the plane-axis
                           // component is mu_axis times the partial sum, not stored
  int32_t frame[3];        // grid axis (0 x, 1 y, 2 z) of cols, rows and the plane axis
  int32_t pad2;
  double tol;              // > 0: laps stop when the last plane changes by <= tol of its largest
                           // intensity (laps is then the largest count); 0: always laps
  int64_t gbuf_off;        // tol: element offset of the previous last plane D [row][col][slot]
  int64_t tolw_off;        // tol: 64-bit word offset of [laps][3] (max change, max intensity,
                           // strips arrived), zeroed by every call
  int64_t n_cells;         // cells of the box
  int64_t xbuf_off;        // 64-bit-word offset of the neighbour exchange buffer
  int64_t it_off;          // element offset of this band's I_top block in the box I_top
  int64_t itp, itr, itc;   // I_top strides for (plane, row, col)
  int64_t it_ray;          // I_top stride between up rays (ny * nx)
  int64_t dstore_off;      // element offset of the stored D of every plane [u][slot][row][col]
  int32_t n_unrolled;      // planes u of the unrolled sweep (u = 0 first plane after the ghost,
                           // or the boundary plane when planes are z)
  int32_t gh_M;            // warm start: max(nx, ny), the row length of a ghost plane
  int32_t nblk[3];         // subdomain decomposition: blocks along cols, rows and planes (all 1
                           // when the box is not divided)
  int32_t iters;           // decomposed box: its iteration count (n_iter)
  int64_t dfield_off;      // decomposed box: element offset of this task's D of every slot and
                           // cell for the two iteration parities [2][slot][plane][row][col]
  int64_t btol_off;        // decomposed box with tol: 64-bit word offset of the box's per-
                           // iteration maxima [iterations][2] (change, intensity)
  int64_t gh_off;          // warm start: element offset of this band's ghost planes
                           // (band * nrays * nz * gh_M); a slot's ray r adds r * nz * gh_M
  double pl_a, pl_b;       // boundary-plane value D = pl_a * S + pl_b (z_planes)
  double bu_a, bu_b;       // boundary row 0 of even slots (rows are z, mu_z > 0)
  double bd_a, bd_b;       // boundary row n_rows-1 of odd slots (rows are z, mu_z < 0)
  TaskRay ray[kMaxRaysPerTask];
};

// Reverse sweep of one task, for the adjoint: two slot-pair passes (slots 0,
// 2 and slots 1, 3), each a persistent strip sweep like the forward one,
// planes in reverse order.  A pass's strips exchange their edge rows through
// a ring of kRevRing steps per strip: ring[strip][kRevRing][2 slots][3][col]
// [64-bit words], followed by one progress word (int32) per strip.
constexpr int kRevRing = 8;
constexpr int64_t rev_ring_words(int strips, int cols, int words) {
  return (int64_t)strips * kRevRing * 6 * cols * words;
}

struct AdjTask {
  int32_t task;       // index into the Task table (AdjTask i < ntasks is the first pass of
                      // Task i; the second passes follow the ntasks)
  int32_t u_init;     // last unrolled plane of the reverse: -1 (ghost plane) or 0
  int32_t strips;     // strips of the reverse launch's rows (rev_rows of its width)
  int32_t nparts;     // gradient partials per quantity: 2, one per pass
  int32_t part;       // this pass's slot parity (slots part and part + 2)
  int32_t pad;
  int64_t xbuf_off;   // 64-bit word offset of the pass's exchange ring and progress words
  int64_t gs_off;     // Real offset of this task's dL/dS partials [part][task array layout]
  int64_t gc_off;     // Real offset of this task's dL/dchi partials [part][task array layout]
  int64_t seed_off;   // Real offset of the band's seed in the task array layout
};

struct RevArgs {
  char* ws;
  const Task* tasks;
  const AdjTask* atasks;
  const int32_t* queue;  // [first ticket, AdjTask index] per task, longest first
  int32_t ntasks;
  int32_t total_strips;
  int64_t timeout_ticks;
  int32_t wclass;                // ticket counter of this launch (WsHeader::ticket_rev)
  int32_t pad;
  const void* gItop[kMaxBoxes];  // per box, [nbands][n_up][ny][nx] or null
  const void* S[kMaxBoxes];      // per box, [nbands][N]
};

struct BoxPtrs {
  const void* kappa;
  const void* rho;
  const void* S;
  double* Q;
  void* J;
  void* I_top;
  double* F;   // [3][N] flux vector, or null
  double* QF;  // [N] its divergence heating, or null
  const void* gin;  // warm start: initial ghost planes [nbands][nrays][nz][max(nx, ny)], or null
  void* gout;       // the final ghost planes (same layout), or null
};

// Per-box geometry for the prep and reduce kernels.
struct BoxGeo {
  int32_t nx, ny, nz, nbands;
  int32_t task0;           // first task of this box (tasks of a box are contiguous, band-major)
  int32_t tasks_per_band;
  int32_t n_up;
  int32_t pad;
  int64_t chi_off;         // workspace element offset of chi [nbands][N]
  int64_t chiT_off;        // chi^T [nbands][nx][nz][ny]
  int64_t sT_off;          // S^T   [nbands][nx][nz][ny]
  double qweight[16];
  double msum[3];          // sum_r w_r mu_r (the flux of an isotropic unit intensity / 4 pi)
  double dx, dy, dz;       // grid spacing (flux divergence)
  double wsum1;            // sum_r w_r - 1: J_b = (1 + wsum1) S_b + sum_r w_r D_r (0 for
                           // normalised weights, then the term vanishes exactly)
};

// Forward sweep launches of one call: one per workgroup width (padded columns).
constexpr int kMaxWidths = kMaxCols / 64;

// Workspace header (first 256 bytes).
struct WsHeader {
  int32_t status;                 // 0, or after a wait timed out: 1 forward neighbour, 2 reverse neighbour, 3 lap end
  int32_t nonfinite;              // set by rts_check_inputs' scan when an input is not finite
  int32_t pad0[2];
  int32_t ticket[kMaxWidths];     // work-queue counter of each forward sweep launch
  int32_t ticket_rev[kMaxWidths]; // work-queue counter of each reverse sweep launch
  int32_t pad[28];
};
static_assert(sizeof(WsHeader) == 256, "workspace header is 256 bytes");

// Scattering with Gauss-Seidel source updates (rts_gs_*): one group of rays
// sharing the dominant axis and its direction (one sweep task), in the natural
// [z][y][x] layout.  Slot k's upwind corners are offset by -sea along the
// first in-plane axis ea and by -seb along the second, eb (ea < eb).
struct GsRay {
  double fa, fb;    // upwind fractions along ea and eb
  double hds;       // ds / 2
  double w;         // quadrature weight (0 for an unused slot)
  int32_t sea, seb; // +1 / -1
  int32_t up;       // mu_z > 0
  int32_t itop;     // index among the rays with mu_z > 0, or -1
  int32_t used;     // a ray occupies the slot
  int32_t pad;
};
struct GsGroup {
  int32_t axis, sa; // dominant axis and direction
  int32_t ea, eb;   // in-plane axes
  int32_t laps;     // n_iter for x or y, 1 for z
  int32_t pad;
  double wsum;      // sum of the group's weights
  GsRay ray[kMaxRaysPerTask];
};
struct GsArgs {
  char* ws;
  const GsGroup* groups;  // in the workspace
  int32_t ngroups, nbands;
  int32_t nx, ny, nz;
  int32_t bot, top;       // rts_bot_bc, rts_top_bc
  int32_t pad;
  double ibot;
  int64_t N;
  int64_t chi_off;        // workspace element offsets (double): chi [B][N]
  int64_t s_off;          // S state [B][N]
  int64_t j_off;          // J state [B][N]
  int64_t p_off;          // group contributions [G][B][N]
  int64_t l_off;          // local operator [B][N]
  int64_t i_off;          // every group's intensities [group][slot][B][N], each [N] block in the
                          // group's plane layout [plane][eb][ea]
  int64_t chit_off;       // chi and the iteration's S in the [x][z][y] layout [B][N] (the
  int64_t st_off;         // x-dominant groups read these: their planes are contiguous there)
  const double* B;        // thermal source [B][N] (the caller's S input)
  const double* eps;      // [B][N]
  double qw[16];          // band weights of Q
  double* Q;
  double* J;              // or null
  double* I_top;          // or null
  double* S;              // final source function, or null
};

// One iteration of a decomposed solve (rts_block_sweep): every (task, block).
struct BlockArgs {
  char* ws;
  const Task* tasks;       // in the workspace
  int32_t ntasks;
  int32_t iter;            // iteration 0, 1, ... (tasks of boxes with fewer iterations return)
  BoxPtrs box[kMaxBoxes];
};

struct SweepArgs {
  char* ws;                // workspace base
  const Task* tasks;       // in the workspace
  const int32_t* queue;    // [ntasks][2]: (first ticket, task index), ascending tickets
  int32_t ntasks;
  int32_t total_strips;
  int64_t timeout_ticks;   // s_memrealtime ticks before a wait gives up
  int32_t store_d;         // also store D of every plane (forward pass of the adjoint)
  int32_t flux;            // also write the flux partials sum_r w_r mu_r D_r
  int32_t ext;             // launch the extended sweep (flux partials and/or tolerance laps)
  int32_t wclass;          // ticket counter of this launch (WsHeader::ticket)
  BoxPtrs box[kMaxBoxes];
};

}  // namespace rts
