// gfx950 kernels of the short-characteristics radiation transport solve (librts)
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
//
// This header holds the device-side helpers every kernel translation unit
// shares: the constant and global address-space casts, device-coherent loads
// and stores, the LDS barrier, the tagged edge-row words and the
// linear-source weight functions.  The kernels are in rts_sweep.hpp (forward
// sweep), rts_reverse.hpp (reverse sweep) and rts_misc.hip (the rest).
#pragma once
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

// Raw buffer access: a uniform 128-bit resource for a base address (4 GiB
// range, 32-bit data format), a per-lane 32-bit byte offset and a uniform
// byte offset.  No per-lane 64-bit address is formed or kept, so a load costs
// one VGPR for its data (global instructions with a per-lane address let the
// compiler hoist a 64-bit address pair per array and per row out of a loop).
typedef __amdgpu_buffer_rsrc_t Rsrc;
__device__ inline Rsrc rts_rsrc(const void* base) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), 0, -1, 0x00020000);
}
__device__ inline float buf_ld(Rsrc r, float*, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
__device__ inline double buf_ld(Rsrc r, double*, uint32_t voff, uint32_t soff) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <class Real>
__device__ inline Real buf_load(Rsrc r, uint32_t voff, uint32_t soff) {
  return buf_ld(r, (Real*)nullptr, voff, soff);
}
__device__ inline void buf_store(Rsrc r, uint32_t voff, uint32_t soff, float v) {
  __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, voff, soff, 0);
}
__device__ inline void buf_store(Rsrc r, uint32_t voff, uint32_t soff, double v) {
  typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
  __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, voff, soff, 0);
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


// c = (1 - e)/x of the linear-source step, e = exp(-x), by its closed form
// or by its power series where 1 - e cancels.  FP32 takes xs = x log2(e) (the
// factor is folded into the scaled opacities) so that e is one v_exp_f32; the
// switch is at x = 0.094, where the closed form's error from the rounding of
// e (one ulp of e over 1 - e, 6.6e-7 relative) and the truncation of a series
// of four terms (x^4/120, 6.5e-7) balance.  FP64 takes xs = x, the switch at
// 0.1 and 11 terms.
__device__ inline float rts_exp_step(float xs) { return __builtin_amdgcn_exp2f(-xs); }
__device__ inline double rts_exp_step(double x) { return exp(-x); }
__device__ inline bool rts_small_step(float xs) { return xs < 0.094f * 1.4426950408889634f; }
__device__ inline bool rts_small_step(double x) { return x < 0.1; }
__device__ inline float rts_c_closed(float xs, float e) {
  // (1 - e) log2(e) / xs, the factor taken into one fma
  constexpr float l2e = 1.4426950408889634f;
  return fmaf(-l2e, e, l2e) * __builtin_amdgcn_rcpf(xs);
}
__device__ inline double rts_c_closed(double x, double e) { return (1.0 - e) / x; }
__device__ inline float rts_c_series(float xs) {
  // sum_{n=0}^{3} (-x)^n / (n+1)!  with x = xs ln2
  constexpr float ln2 = 0.69314718055994531f;
  constexpr float a1 = -ln2 / 2.f, a2 = ln2 * ln2 / 6.f, a3 = -ln2 * ln2 * ln2 / 24.f;
  return fmaf(fmaf(fmaf(xs, a3, a2), xs, a1), xs, 1.f);
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


}  // namespace rts
