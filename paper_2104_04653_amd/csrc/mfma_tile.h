// FP64 16 x 16 register tiles for the matrix cores of gfx950, shared by the
// local-solve kernels.
//
// A tile lives in the output layout of v_mfma_f64_16x16x4f64, measured on
// the device: lane l = c + 16 g (c = l & 15, g = l >> 4) holds rows g, g+4,
// g+8, g+12 of column c in its four registers (row 4 v + g in register v).
// Passing a tile's registers as the A operand of the four K = 4 steps
// (element kk of the lane's registers in step kk, K index k = 4 kk + g) and
// another tile's as the B operand computes A^T B: for a symmetric A (an
// inverse Schur block) that is A B, with no data moving between lanes.
#pragma once

#include <hip/hip_runtime.h>

namespace mrcm {
namespace tile {

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline double readlane_d(double x, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffu), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

__device__ inline d4 mfma(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// 1/p from the hardware reciprocal estimate (relative error below 5e-8)
// and one Newton step, which squares it (below 3e-15), in place of the IEEE
// division sequence: every solve with these inverse blocks is refined
// against the exact matrix, so their last digits do not reach the results
__device__ inline double recip(double p) {
  const double r = __builtin_amdgcn_rcp(p);
  return fma(r, fma(-p, r, 1.0), r);
}

// value of lane K of each 16-lane row (one 64-bit DPP row_newbcast move;
// every lane has a valid source, so bound_ctrl only spares the compiler the
// copy of an "old" value into the destination first)
template <int K>
__device__ inline double row_bcast(double x) {
  return __longlong_as_double(
      __builtin_amdgcn_update_dpp(0LL, __double_as_longlong(x), 0x150 + K, 0xF, 0xF, true));
}

// min(m, p) for pivot tracking, with p uniform (a scalar register): the
// plain v_min_f64, without the quieting of NaN operands that fmin adds (a
// NaN pivot is caught by the pnan accumulator instead)
__device__ inline double pivot_min(double m, double p) {
  double r;
  asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(m), "s"(p));
  return r;
}

// One Gauss-Jordan sweep with pivot K on a tile in the output layout: the
// pivot column (row 4 v + g, column K) comes from lane K of the lane's own
// 16-lane row, the pivot row (row K, column c) from lane c of row K % 4.
// Column K is replaced by -pcol / p rather than updated: its old value is
// multiplied by 0 (one multiply per register instead of a two-instruction
// select).  Pivot health is accumulated without branches: pmin = min of
// the pivots, pnan = sum of pivot * 0 (NaN once a pivot was not finite).
template <int K>
__device__ inline void gj_sweep(d4& s, int c, int g, double& pmin, double& pnan) {
  constexpr int kv = K >> 2, kg = K & 3;
  const double p = readlane_d(s[kv], K + 16 * kg);
  const double prow = __shfl(s[kv], c + 16 * kg);
  double pcol[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) pcol[v] = row_bcast<K>(s[v]);
  pmin = pivot_min(pmin, p);
  pnan = fma(p, 0.0, pnan);
  const double ip = recip(p);
  const double b = (c == K) ? ip : prow * ip;      // new row K
  const double keep = (c == K) ? 0.0 : 1.0;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double nv = fma(-pcol[v], b, s[v] * keep);
    s[v] = (v == kv && g == kg) ? b : nv;
  }
}

template <int K>
struct GJ16 {
  static __device__ inline void run(d4& s, int c, int g, double& pmin, double& pnan) {
    gj_sweep<K>(s, c, g, pmin, pnan);
    GJ16<K + 1>::run(s, c, g, pmin, pnan);
  }
};
template <>
struct GJ16<16> {
  static __device__ inline void run(d4&, int, int, double&, double&) {}
};

// Health of all pivots of a kernel's Gauss-Jordan inversions, accumulated
// without branches (a per-pivot test would keep every pivot live until the
// kernel's final status write).
struct PivotCheck {
  double pmin = 1.0, pnan = 0.0;
  __device__ bool bad() const { return !(pmin > 0.0) || pnan != 0.0; }
};

// In-place inverse of the SPD tile s (output layout) by Gauss-Jordan sweeps.
__device__ inline d4 gauss_jordan16(d4 s, int c, int g, PivotCheck& pc) {
  GJ16<0>::run(s, c, g, pc.pmin, pc.pnan);
  // materialise the accumulators here, so that the pivots die with the sweep
  asm volatile("" : "+v"(pc.pmin), "+v"(pc.pnan));
  return s;
}

// acc + A^T B for tiles A, B in the output layout (A B for a symmetric A)
__device__ inline d4 mm_tn(const d4& A, const d4& B, d4 acc) {
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) acc = mfma(A[kk], B[kk], acc);
  return acc;
}

}  // namespace tile
}  // namespace mrcm
