// FP64 solve of the MRCM interface system (paper, section 3, eq. (mrc2))
// on gfx950.
//
// The interface system is the sum over subdomains of the symmetric
// per-subdomain blocks written by the local kernel (rows of the
// pressure-continuity equations negated).  The sum is symmetric
// quasi-definite: its pressure-pressure part is negative semidefinite and
// its flux-flux part positive definite, so an elimination without pivoting
// exists for any ordering.  It is eliminated with a nested-dissection tree
// over the subdomain grid: boxes of subdomains are split in two along their
// longer side; a node gathers its two children's Schur complements
// ("extend-add", a deterministic gather), eliminates the interface unknowns
// on the line that separates the children, and passes the Schur complement
// on the box boundary to its parent.  The leaves are the subdomain blocks
// themselves, so the global matrix is never formed.
//
// Fronts of up to SMALL_FRONT unknowns are gathered and eliminated by one
// work-group in registers.  Larger fronts (the nodes near the root) are
// eliminated in global memory by a right-looking blocked LU, one launch
// per panel of PANEL_NB columns: the trailing update A22 -= A21 (A11^-1 A12)
// in 64 x 64 tiles on the FP64 matrix cores, with the next panel's
// diagonal block updated and inverted by a work-group of its own (two
// 16 x 16 Gauss-Jordan inversions without pivoting, which the
// quasi-definite structure allows, joined by a Schur complement).  The first
// panel's launch also assembles the fronts: its work-groups read their
// operands straight from the children and write the assembled front.
// Back substitution runs top down, one work-group per node.
#include "mrcm_internal.h"

#include <math.h>

namespace mrcm {

namespace {

constexpr int NT = 256;

// entry of a front from its two children (extend-add).  Both children's
// entries are loaded unconditionally (from the start of the tree buffer
// when the unknown is not the child's) and selected afterwards: a branch
// around each load would make every load wait for the one before it.
__device__ inline double gather_entry(const NodeDesc& nd, const double* tree, int2 ma, int2 mb,
                                      bool rhs) {
  const bool u0 = ma.x >= 0 && (rhs || mb.x >= 0), u1 = ma.y >= 0 && (rhs || mb.y >= 0);
  const long long i0 =
      u0 ? nd.c_off[0] + (long long)ma.x * nd.c_ld[0] + (rhs ? nd.c_rhs[0] : mb.x) : 0;
  const long long i1 =
      u1 ? nd.c_off[1] + (long long)ma.y * nd.c_ld[1] + (rhs ? nd.c_rhs[1] : mb.y) : 0;
  const double x0 = tree[i0], x1 = tree[i1];
  return (u0 ? x0 : 0.0) + (u1 ? x1 : 0.0);
}

// double-double accumulation: (hi, lo) += v, and (hi, lo) -= a b
__device__ inline void two_sum(double& hi, double& lo, double v) {
#pragma clang fp contract(off)
  const double s = hi + v, bb = s - hi;
  lo += (hi - (s - bb)) + (v - bb);
  hi = s;
}
__device__ inline void two_prod_sub(double& hi, double& lo, double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b, pe = fma(a, b, -p);
  two_sum(hi, lo, -p);
  lo -= pe;
}

// 2-D thread map used by the element loops below (no integer division):
// 32 columns x 8 rows per pass.
constexpr int TXN = 32, TYN = NT / TXN;

// A front of up to SMALL_FRONT unknowns, eliminated in registers: thread
// (tx, ty) holds the entries of rows ty + TYN i and columns tx + TXN j
// (column n: the rhs), RI x CJ of them, for the whole elimination.  At
// pivot k the holders of row k and of column k put them in LDS (double
// buffered, so one barrier per pivot), and every thread updates its own
// entries: F[a][k] becomes the multiplier F[a][k] / F[k][k], and
// F[a][b] -= F[a][k] F[k][b] for a, b > k.  The result (U in the
// eliminated rows, multipliers below them, the Schur complement and its
// rhs in the trailing block) is stored row-major, n x (n + 1).
template <int RI, int CJ>
__global__ void __launch_bounds__(NT) front_small_kernel(const NodeDesc* nodes, double* tree,
                                                         const int2* maps, int* status,
                                                         unsigned long long* stamp) {
  if (stamp && blockIdx.x == 0 && threadIdx.x == 0) stamp_now(stamp);
  __shared__ int2 mp[SMALL_FRONT];
  __shared__ double prow[2][SMALL_FRONT + 1], pcol[2][SMALL_FRONT];
  const NodeDesc nd = nodes[blockIdx.x];   // this level's fronts, one per work-group
  const int n = nd.n, s = nd.s, ld = n + 1;
  const int tid = threadIdx.x, tx = tid % TXN, ty = tid / TXN;
  for (int a = tid; a < n; a += NT) mp[a] = maps[nd.map_off + a];
  __syncthreads();
  // every entry's loads in flight together: unconditional, from clamped
  // indices, entries outside the front dropped afterwards
  double R[RI][CJ];
#pragma unroll
  for (int i = 0; i < RI; ++i) {
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      const int a = ty + TYN * i, b = tx + TXN * j;
      const int ac = min(a, n - 1), bc = min(b, n);
      const double x = gather_entry(nd, tree, mp[ac], bc < n ? mp[bc] : mp[ac], bc == n);
      R[i][j] = (a < n && b <= n) ? x : 0.0;
    }
  }
  // the pivot loop is written with selects, not branches: per-entry
  // branches compile to hundreds of exec-mask blocks per pivot
  bool bad = false;
  for (int k = 0; k < s; ++k) {
    const int bf = k & 1;
    const int ik = k / TYN, jk = k / TXN;   // register row / column that hold pivot row / column
    if (ty == k % TYN) {
#pragma unroll
      for (int j = 0; j < CJ; ++j) {
        double v = R[0][j];
#pragma unroll
        for (int i = 1; i < RI; ++i) v = i == ik ? R[i][j] : v;
        if (tx + TXN * j <= n) prow[bf][tx + TXN * j] = v;
      }
    }
    if (tx == k % TXN) {
#pragma unroll
      for (int i = 0; i < RI; ++i) {
        double v = R[i][0];
#pragma unroll
        for (int j = 1; j < CJ; ++j) v = j == jk ? R[i][j] : v;
        if (ty + TYN * i < n) pcol[bf][ty + TYN * i] = v;
      }
    }
    __syncthreads();
    const double piv = prow[bf][k];
    if (piv == 0.0 || !isfinite(piv)) bad = true;
    const double ip = 1.0 / piv;
    double pr[CJ];
#pragma unroll
    for (int j = 0; j < CJ; ++j) pr[j] = prow[bf][min(tx + TXN * j, n)];
#pragma unroll
    for (int i = 0; i < RI; ++i) {
      const int a = ty + TYN * i;
      const double f = pcol[bf][min(a, n - 1)] * ip;
      const bool below = a > k && a < n;
#pragma unroll
      for (int j = 0; j < CJ; ++j) {
        const int b = tx + TXN * j;
        const double upd = R[i][j] - f * pr[j];
        const double nv = b == k ? f : ((b > k && b <= n) ? upd : R[i][j]);
        R[i][j] = below ? nv : R[i][j];
      }
    }
  }
  double* out = tree + nd.f_off;
#pragma unroll
  for (int i = 0; i < RI; ++i) {
#pragma unroll
    for (int j = 0; j < CJ; ++j) {
      const int a = ty + TYN * i, b = tx + TXN * j;
      if (a < n && b <= n) out[(long long)a * ld + b] = R[i][j];
    }
  }
  if (bad && tid == 0) atomicOr(status, ST_IFACE_PIVOT);
}

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ inline d4 mfma64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

__device__ inline double readlane_d(double x, int lane) {
  const unsigned long long u = (unsigned long long)__double_as_longlong(x);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u & 0xffffffffu), lane);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), lane);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// value of lane K of each 16-lane row (one 64-bit DPP row_newbcast move;
// every lane has a valid source, so bound_ctrl only spares the copy of an
// "old" value into the destination)
template <int K>
__device__ inline double row_bcast(double x) {
  return __longlong_as_double(
      __builtin_amdgcn_update_dpp(0LL, __double_as_longlong(x), 0x150 + K, 0xF, 0xF, true));
}

// min(m, |p|) for pivot tracking, p uniform: the plain v_min_f64 (a NaN
// pivot is caught by the pnan accumulator, so no quieting is needed)
__device__ inline double pivot_min_abs(double m, double p) {
  double r;
  asm("v_min_f64 %0, %1, |%2|" : "=v"(r) : "v"(m), "s"(p));
  return r;
}

// One Gauss-Jordan sweep with pivot K on a 16 x 16 tile held by one
// wavefront in the MFMA output layout (lane c + 16 g holds rows 4 v + g of
// column c in s[v]), no pivoting: the pivot column comes from lane K of the
// lane's own 16-lane row, the pivot row from lane c + 16 (K % 4).
// Pivot health is accumulated without branches: pmin = min |pivot|, pnan =
// sum of pivot * 0 (NaN once a pivot was not finite).
template <int K>
__device__ inline void gj16_sweep(d4& s, int c, int g, double& pmin, double& pnan) {
  constexpr int kv = K >> 2, kg = K & 3;
  const double p = readlane_d(s[kv], K + 16 * kg);
  const double prow = __shfl(s[kv], c + 16 * kg);
  double pcol[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) pcol[v] = row_bcast<K>(s[v]);
  pmin = pivot_min_abs(pmin, p);
  pnan = fma(p, 0.0, pnan);
  double ip = __builtin_amdgcn_rcp(p);              // reciprocal estimate, two Newton steps
  ip = fma(ip, fma(-p, ip, 1.0), ip);
  ip = fma(ip, fma(-p, ip, 1.0), ip);
  const double b = (c == K) ? ip : prow * ip;      // new row K
  const double keep = (c == K) ? 0.0 : 1.0;        // column K is replaced, not updated
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const double nv = fma(-pcol[v], b, s[v] * keep);
    s[v] = (v == kv && g == kg) ? b : nv;
  }
}

template <int K>
struct GJ16 {
  static __device__ inline void run(d4& s, int c, int g, double& pmin, double& pnan) {
    gj16_sweep<K>(s, c, g, pmin, pnan);
    GJ16<K + 1>::run(s, c, g, pmin, pnan);
  }
};
template <>
struct GJ16<16> {
  static __device__ inline void run(d4&, int, int, double&, double&) {}
};

// In-place inverse of a 16 x 16 tile (output layout) by Gauss-Jordan sweeps;
// bad is set if a pivot was zero or not finite.
__device__ inline d4 gj16(d4 s, int c, int g, bool& bad) {
  double pmin = 1.0, pnan = 0.0;
  GJ16<0>::run(s, c, g, pmin, pnan);
  if (!(pmin > 0.0) || pnan != 0.0) bad = true;
  return s;
}

// Inverse of the symmetric PANEL_NB x PANEL_NB diagonal block in S (LDS;
// identity-padded beyond the panel width; only its upper triangle of 16 x 16
// tiles is read), by one wavefront, written to `out` row-major.  With
// A = [P Q; Q^T B]:  X = P^-1 Q,  C = B - Q^T X,  and
// A^-1 = [P^-1 + X C^-1 X^T, -X C^-1; -C^-1 X^T, C^-1].
// The products run on the matrix cores with the K index of step kk taken as
// 4 kk + g, so that a symmetric left factor and any right factor in the
// output layout are read from the lane's own registers; X^T as a left
// factor comes from one transpose through `T`.  The pivots of the two 16 x 16
// inversions are the pivots of an LU factorisation of A.
// The result goes to out with row stride LDO; out may be S itself (stride
// PANEL_NB + 1): S is read in full before anything is written.  A block
// of width nb <= 16 is [P 0; 0 I]: its inverse [P^-1 0; 0 I] takes one
// 16 x 16 inversion.
template <int LDO>
__device__ void inv32_wave(const double (*S)[PANEL_NB + 1], double (*T)[17], double* out,
                           bool& bad, int nb) {
  static_assert(PANEL_NB == 32, "two 16 x 16 tiles per side");
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  d4 P, Q, B;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * v + g;
    P[v] = S[r][c];
    Q[v] = S[r][16 + c];
    B[v] = S[16 + r][16 + c];
  }
  const d4 z = {0.0, 0.0, 0.0, 0.0};
  const d4 Pi = gj16(P, c, g, bad);
  if (nb <= 16) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int r = 4 * v + g;
      out[r * LDO + c] = Pi[v];
      out[(16 + r) * LDO + c] = 0.0;
      out[c * LDO + 16 + r] = 0.0;
      out[(16 + r) * LDO + 16 + c] = r == c ? 1.0 : 0.0;
    }
    return;
  }
  d4 X = z;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) X = mfma64(Pi[kk], Q[kk], X);          // P^-1 Q
  d4 QX = z;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) QX = mfma64(Q[kk], X[kk], QX);         // Q^T X
  const d4 Ci = gj16(B - QX, c, g, bad);
#pragma unroll
  for (int v = 0; v < 4; ++v) T[4 * v + g][c] = X[v];
  __builtin_amdgcn_wave_barrier();
  d4 Xt;                                                                // X[c][4 kk + g]
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) Xt[kk] = T[c][4 * kk + g];
  d4 L = z;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) L = mfma64(Ci[kk], Xt[kk], L);         // C^-1 X^T
  d4 U = Pi;
#pragma unroll
  for (int kk = 0; kk < 4; ++kk) U = mfma64(Xt[kk], L[kk], U);          // P^-1 + X C^-1 X^T
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int r = 4 * v + g;
    out[r * LDO + c] = U[v];
    out[(16 + r) * LDO + c] = -L[v];
    out[c * LDO + 16 + r] = -L[v];
    out[(16 + r) * LDO + 16 + c] = Ci[v];
  }
}

__device__ inline double* panel_inv(double* inv, const NodeDesc& nd, int k0) {
  return inv + nd.inv_off + (long long)(k0 / PANEL_NB) * PANEL_NB * PANEL_NB;
}

// Trailing update of panel k0 for one 64 x 64 tile of a blocked front,
// A22 -= A21 W with W = A11^-1 A12 formed for the tile's columns, both
// products on v_mfma_f64_16x16x4f64 (lane c + 16 g holds rows 4 v + g of
// column c of a 16 x 16 result; operand A[i][k] from lane i + 16 k, B[k][j]
// from lane j + 16 k).  The panel rows and columns themselves are left as
// they were at the start of the panel (back substitution applies A11^-1 to
// them), so tiles never write what other tiles read.
// The next panel's diagonal block is the critical path of the elimination:
// it is updated and inverted by an item of its own (kind 2, a 32 x 32 tile
// with one 16 x 16 product tile per wavefront, dispatched first), and the
// 64 x 64 tile that contains it (kind 1) leaves it out.
// FIRST: the first panel, fused with the assembly of the front from its
// children (extend-add: a parent's system is the sum of its children's
// Schur complements over the shared unknowns).  Every item reads the
// entries it needs straight from the children, inverts the panel's
// diagonal block itself (one wavefront, in LDS), and writes its tile of the
// assembled and updated front; the tiles next to the panel also store the
// panel's rows and columns as assembled.  Kind 3 items do that for a front
// without trailing rows (a 64-column stretch of the panel rows; the one at
// (0, 0) also stores the diagonal block's inverse).
template <bool FIRST>
__global__ void __launch_bounds__(NT) front_update_kernel(const NodeDesc* nodes,
                                                          const PanelItem* items, int k0,
                                                          double* tree, const int2* maps,
                                                          double* inv, int* status,
                                                          unsigned long long* stamp) {
  if (stamp && blockIdx.x == 0 && threadIdx.x == 0) stamp_now(stamp);
  __shared__ double Dv[PANEL_NB][PANEL_NB + 1];   // A11^-1; then the next diagonal block
  __shared__ double As[TILE][PANEL_NB + 1];       // A21 rows of the tile
  __shared__ double Bs[PANEL_NB][TILE + 1];       // A12 columns of the tile; then W = A11^-1 A12
  __shared__ double Tt[16][17];
  __shared__ int2 mr[TILE], mc[TILE], mk[PANEL_NB];   // FIRST: maps of rows, columns, panel
  static_assert(TILE == 64 && PANEL_NB == 32 && NT == 256, "tile shape of the MFMA mapping");
  const PanelItem it = items[blockIdx.x];   // carries the front's fields: one load round
  const int kind = it.pad;                  // 0: tile, 1: tile without its leading diagonal
                                            // block, 2: that block alone (then inverted),
                                            // 3 (FIRST): panel rows or columns, stored
  const int n = it.n, ld = n + 1;
  const int nb = min(PANEL_NB, it.s - k0);
  const int nb1 = min(PANEL_NB, it.s - (k0 + nb));   // next panel's width (kinds 1, 2)
  double* F = tree + it.f_off;
  const double* iv = inv + it.inv_off + (long long)(k0 / PANEL_NB) * PANEL_NB * PANEL_NB;
  const int t = threadIdx.x;
  const int r0 = it.i0, c0 = it.j0;
  int rows = kind == 2 ? nb1 : min(TILE, n - r0), cols = kind == 2 ? nb1 : min(TILE, ld - c0);
  // a tile followed by the rhs column alone also updates that column (plain
  // FMAs instead of a work-group of its own)
  const bool xr = (kind == 0 || kind == 1) && ld - c0 == TILE + 1;
  const int w = t >> 6, lane = t & 63, c = lane & 15, g = lane >> 4;
  NodeDesc nd;
  if constexpr (FIRST) {
    nd = nodes[it.node];
    const int2* mp = maps + nd.map_off;
    if (t < TILE) mr[t] = mp[min(r0 + t, n - 1)];
    else if (t < 2 * TILE) mc[t - TILE] = mp[min(c0 + t - TILE, n - 1)];   // column n: the rhs
    else if (t < 2 * TILE + PANEL_NB) mk[t - 2 * TILE] = mp[min(t - 2 * TILE, n - 1)];
    __syncthreads();
  }
  // entry (r0 + i, c0 + j) of the front at the start of the panel
  auto a22_at = [&](int i, int j) -> double {
    if constexpr (FIRST) return gather_entry(nd, tree, mr[i], mc[j], c0 + j == n);
    else return F[(long long)(r0 + i) * ld + c0 + j];
  };
  if constexpr (FIRST) {
    if (kind == 3) {
      if (r0 == 0) rows = nb; else cols = nb;   // panel rows / panel columns
      constexpr int PER = TILE * TILE / NT;
      double v[PER];
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = t + NT * q, i = e / TILE, j = e % TILE;
        const double x = a22_at(min(i, rows - 1), min(j, cols - 1));
        v[q] = (i < rows && j < cols) ? x : 0.0;
      }
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int e = t + NT * q, i = e / TILE, j = e % TILE;
        if (i < rows && j < cols) F[(long long)(r0 + i) * ld + c0 + j] = v[q];
      }
      if (r0 == 0 && c0 == 0) {
        constexpr int PD = PANEL_NB * PANEL_NB / NT;
        double xd[PD];
#pragma unroll
        for (int q = 0; q < PD; ++q) {
          const int e = t + NT * q, i = min(e / PANEL_NB, nb - 1), k = min(e % PANEL_NB, nb - 1);
          xd[q] = gather_entry(nd, tree, mk[i], mk[k], false);
        }
#pragma unroll
        for (int q = 0; q < PD; ++q) {
          const int e = t + NT * q, i = e / PANEL_NB, k = e % PANEL_NB;
          Dv[i][k] = (i < nb && k < nb) ? xd[q] : (i == k ? 1.0 : 0.0);
        }
        __syncthreads();
        if (t < 64) {
          bool bad = false;
          inv32_wave<PANEL_NB>(Dv, Tt, inv + it.inv_off, bad, nb);
          if (bad) atomicOr(status, ST_IFACE_PIVOT);
        }
      }
      return;
    }
  }
  // the rhs column after the tile (xr): A22 rows in wave 0, panel rows in
  // the first half of wave 1 (loaded either way, used only with xr)
  double xrv;
  {
    const int i = min(t < 64 ? t : t - 64, t < 64 ? rows - 1 : nb - 1);
    const int row = t < 64 ? r0 + i : k0 + i;
    if constexpr (FIRST) xrv = gather_entry(nd, tree, t < 64 ? mr[i] : mk[i], mk[0], true);
    else xrv = F[(long long)row * ld + n];
  }
  // the panel operands: A11 (first panel: gathered, identity beyond its
  // width, and inverted in place below; else its stored inverse), and the
  // A21 rows and A12 columns of the tile, all loaded before any is stored
  constexpr int PD = PANEL_NB * PANEL_NB / NT, PA = TILE * PANEL_NB / NT;
  double xd[PD], xa[PA], xb[PA];
#pragma unroll
  for (int q = 0; q < PD; ++q) {
    const int e = t + NT * q, i = min(e / PANEL_NB, nb - 1), k = min(e % PANEL_NB, nb - 1);
    if constexpr (FIRST) xd[q] = gather_entry(nd, tree, mk[i], mk[k], false);
    else xd[q] = iv[i * PANEL_NB + k];
  }
#pragma unroll
  for (int q = 0; q < PA; ++q) {
    const int e = t + NT * q, i = min(e / PANEL_NB, rows - 1), k = min(e % PANEL_NB, nb - 1);
    if constexpr (FIRST) xa[q] = gather_entry(nd, tree, mr[i], mk[k], false);
    else xa[q] = F[(long long)(r0 + i) * ld + k0 + k];
  }
#pragma unroll
  for (int q = 0; q < PA; ++q) {
    const int e = t + NT * q, k = min(e / TILE, nb - 1), j = min(e % TILE, cols - 1);
    if constexpr (FIRST) xb[q] = gather_entry(nd, tree, mk[k], mc[j], c0 + j == n);
    else xb[q] = F[(long long)(k0 + k) * ld + c0 + j];
  }
  // this thread's entries of the A22 tile (kind 2: wave w owns the 16 x 16
  // tile (w / 2, w % 2), in a22[0]), issued after the panel operands: a
  // wait for a load waits for every load issued before it, and A22 is used
  // last, so these stay in flight through the inversion and the products.
  // Like all loads here they are unconditional, from indices clamped into
  // the block, and entries outside it are dropped afterwards: a branch
  // around a load would make each load wait for the previous one.
  double a22[4][4];
  const bool k2 = kind == 2;
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // kind 2 reads its one tile four times over: the loads stay unconditional
      const int i = (k2 ? 16 * (w >> 1) : 16 * w) + 4 * v + g, j = (k2 ? 16 * (w & 1) : 16 * tj) + c;
      const double x = a22_at(min(i, rows - 1), min(j, cols - 1));
      a22[tj][v] = (i < rows && j < cols) ? x : 0.0;
    }
  }
#pragma unroll
  for (int q = 0; q < PD; ++q) {
    const int e = t + NT * q, i = e / PANEL_NB, k = e % PANEL_NB;
    Dv[i][k] = (i < nb && k < nb) ? xd[q] : ((FIRST && i == k) ? 1.0 : 0.0);
  }
#pragma unroll
  for (int q = 0; q < PA; ++q) {
    const int e = t + NT * q, i = e / PANEL_NB, k = e % PANEL_NB;
    As[i][k] = (i < rows && k < nb) ? xa[q] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < PA; ++q) {
    const int e = t + NT * q, k = e / TILE, j = e % TILE;
    Bs[k][j] = (k < nb && j < cols) ? xb[q] : 0.0;
  }
  if (t >= 64 && t < 64 + PANEL_NB) Bs[t - 64][TILE] = (xr && t - 64 < nb) ? xrv : 0.0;
  if constexpr (FIRST) {
    // the panel's own rows and columns, as assembled: the first tile row
    // stores the A12 columns it read, the first tile column the A21 rows,
    // the tile at (nb, nb) also A11 and, once inverted, its inverse
    const bool lead = kind != 2 && r0 == nb && c0 == nb;
    if (kind != 2 && c0 == nb) {
#pragma unroll
      for (int q = 0; q < PA; ++q) {
        const int e = t + NT * q, i = e / PANEL_NB, k = e % PANEL_NB;
        if (i < rows && k < nb) F[(long long)(r0 + i) * ld + k] = xa[q];
      }
    }
    if (kind != 2 && r0 == nb) {
#pragma unroll
      for (int q = 0; q < PA; ++q) {
        const int e = t + NT * q, k = e / TILE, j = e % TILE;
        if (k < nb && j < cols) F[(long long)k * ld + c0 + j] = xb[q];
      }
      if (xr && t >= 64 && t - 64 < nb) F[(long long)(t - 64) * ld + n] = xrv;
    }
    if (lead) {
#pragma unroll
      for (int q = 0; q < PD; ++q) {
        const int e = t + NT * q, i = e / PANEL_NB, k = e % PANEL_NB;
        if (i < nb && k < nb) F[(long long)i * ld + k] = xd[q];
      }
    }
    __syncthreads();
    if (t < 64) {
      bool bad = false;
      inv32_wave<PANEL_NB + 1>(Dv, Tt, &Dv[0][0], bad, nb);
      if (lead && bad) atomicOr(status, ST_IFACE_PIVOT);
    }
    if (lead) {
      __syncthreads();
      double* out = inv + it.inv_off;
#pragma unroll
      for (int q = 0; q < PD; ++q) {
        const int e = t + NT * q;
        out[e] = Dv[e / PANEL_NB][e % PANEL_NB];
      }
    }
  }
  __syncthreads();
  if (kind == 2) {
    // the next diagonal block: W and A21 W, one 16 x 16 tile per wave
    const int ti = w >> 1, tj = w & 1;
    d4 wv = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < PANEL_NB / 4; ++q) wv = mfma64(Dv[16 * ti + c][4 * q + g], Bs[4 * q + g][16 * tj + c], wv);
    __syncthreads();   // W replaces A12
#pragma unroll
    for (int v = 0; v < 4; ++v) Bs[16 * ti + 4 * v + g][16 * tj + c] = wv[v];
    __syncthreads();
    d4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < PANEL_NB / 4; ++q) acc = mfma64(As[16 * ti + c][4 * q + g], Bs[4 * q + g][16 * tj + c], acc);
    __syncthreads();   // Dv is reused below
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * ti + 4 * v + g, j = 16 * tj + c;
      double val = (i == j) ? 1.0 : 0.0;   // identity beyond the block's width
      if (i < rows && j < cols) {
        val = a22[0][v] - acc[v];
        F[(long long)(r0 + i) * ld + c0 + j] = val;
      }
      Dv[i][j] = val;
    }
    __syncthreads();
    if (t < 64) {
      bool bad = false;
      inv32_wave<PANEL_NB>(Dv, Tt, inv + it.inv_off + (long long)((k0 + nb) / PANEL_NB) * PANEL_NB * PANEL_NB,
                           bad, nb1);
      if (bad) atomicOr(status, ST_IFACE_PIVOT);
    }
    return;
  }
  {
    // W: 2 x 4 result tiles of 16 x 16, two per wave
    const int ti = w >> 1, tj = 2 * (w & 1);
    d4 a0 = {0.0, 0.0, 0.0, 0.0}, a1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int q = 0; q < PANEL_NB / 4; ++q) {
      const double av = Dv[16 * ti + c][4 * q + g];
      a0 = mfma64(av, Bs[4 * q + g][16 * tj + c], a0);
      a1 = mfma64(av, Bs[4 * q + g][16 * tj + 16 + c], a1);
    }
    double wr = 0.0;   // xr: W of the rhs column, row t
    if (xr && t < PANEL_NB) {
#pragma unroll 8
      for (int m = 0; m < PANEL_NB; ++m) wr = fma(Dv[t][m], Bs[m][TILE], wr);
    }
    __syncthreads();   // W replaces A12
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      Bs[16 * ti + 4 * v + g][16 * tj + c] = a0[v];
      Bs[16 * ti + 4 * v + g][16 * tj + 16 + c] = a1[v];
    }
    if (xr && t < PANEL_NB) Bs[t][TILE] = wr;
  }
  __syncthreads();
  // A21 W: wave w owns rows 16 w .. 16 w + 15 and all four column tiles
  d4 acc[4];
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) acc[tj] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int q = 0; q < PANEL_NB / 4; ++q) {
    const double av = As[16 * w + c][4 * q + g];
#pragma unroll
    for (int tj = 0; tj < 4; ++tj) acc[tj] = mfma64(av, Bs[4 * q + g][16 * tj + c], acc[tj]);
  }
  const int skip = kind == 1 ? nb1 : 0;   // leading diagonal block left to its own item
#pragma unroll
  for (int tj = 0; tj < 4; ++tj) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * w + 4 * v + g, j = 16 * tj + c;
      if (i < rows && j < cols && !(i < skip && j < skip))
        F[(long long)(r0 + i) * ld + c0 + j] = a22[tj][v] - acc[tj][v];
    }
  }
  if (xr && t < rows) {
    double ar = 0.0;
#pragma unroll 8
    for (int k = 0; k < PANEL_NB; ++k) ar = fma(As[t][k], Bs[k][TILE], ar);
    F[(long long)(r0 + t) * ld + n] = xrv - ar;
  }
}

// v - sum of row[m] xl[m] over m = m0, m0 + 8, ... below n, in that
// order.  The row is read CH values at a time, unconditionally from
// clamped indices, so that each chunk is one round of loads in flight.
template <int CH>
__device__ inline double row_dot_sub(double v, const double* row, const double* xl, int m0, int n) {
  for (int mb = m0; mb < n; mb += 8 * CH) {
    double f[CH];
#pragma unroll
    for (int j = 0; j < CH; ++j) f[j] = row[min(mb + 8 * j, n - 1)];
#pragma unroll
    for (int j = 0; j < CH; ++j) {
      const int m = mb + 8 * j;
      const double pr = f[j] * xl[min(m, n - 1)];
      v -= m < n ? pr : 0.0;
    }
  }
  return v;
}

// Back substitution of one front, top down in the tree: x_s from the
// front's eliminated rows and the x_r of its ancestors.
//  classic fronts: row k holds U (upper part) at elimination time k;
//  blocked fronts: the rows of panel p hold the panel-time A12 to the right
//  of the diagonal block, so x_1 = A11^{-1} (b_1 - A12 x_2).
// BLOCKED: the level's fronts are blocked (all of a level's fronts are of
// one kind), a separate instance so that its load registers do not limit
// the occupancy of the many small classic fronts.
template <bool BLOCKED>
__global__ void __launch_bounds__(NT) front_back_kernel(const NodeDesc* nodes, const double* tree,
                                                        const double* inv, const int* dofs,
                                                        const double* rtree, double* x) {
  extern __shared__ double xl[];   // n values: front-local unknowns
  __shared__ double y[PANEL_NB];
  const NodeDesc nd = nodes[blockIdx.x];
  const int n = nd.n, s = nd.s, ld = n + 1;
  const double* F = tree + nd.f_off;
  const int* dof = dofs + nd.dof_off;
  const double* rv = rtree ? rtree + nd.r_off : nullptr;   // rhs vector, else column n
  const int t = threadIdx.x;
  // the separator's own U block (s x s, classic fronts up to US_MAX) goes to
  // LDS with the ancestors' unknowns, so that the triangular solve below
  // reads no global memory
  constexpr int US_MAX = 32;
  __shared__ double Us[US_MAX][US_MAX + 1];
  const bool stage = !BLOCKED && s <= US_MAX;
  if (stage)
    for (int e = t; e < s * s; e += NT) Us[e / s][e % s] = F[(long long)(e / s) * ld + e % s];
  for (int m = s + t; m < n; m += NT) xl[m] = x[dof[m]];
  __syncthreads();
  if constexpr (!BLOCKED) {
    for (int k0 = 0; k0 < s; k0 += NT / 8) {
      const int k = k0 + t / 8, lane = t % 8;
      double v = 0.0;
      if (k < s) {
        const double* row = F + (long long)k * ld;
        const double bk = rv ? rv[k] : row[n];   // in flight with the row's loads
        v = row_dot_sub<8>(v, row, xl, s + lane, n);
        if (lane == 0) v += bk;
      }
      for (int off = 4; off > 0; off >>= 1) v += __shfl_down(v, off, 8);
      if (k < s && lane == 0) xl[k] = v;
    }
    __syncthreads();
    if (stage) {
      // triangular solve by the first wavefront, lane i holding x_i
      if (t < 64) {
        double xi = t < s ? xl[t] : 0.0;
        for (int k = s - 1; k >= 0; --k) {
          const double xk = __shfl(xi, k) / Us[k][k];
          if (t < k) xi -= Us[t][k] * xk;
          if (t == k) xi = xk;
        }
        if (t < s) xl[t] = xi;
      }
      __syncthreads();
    } else {
      for (int k = s - 1; k >= 0; --k) {
        const double xk = xl[k] / F[(long long)k * ld + k];
        __syncthreads();
        for (int i = t; i < k; i += NT) xl[i] -= F[(long long)i * ld + k] * xk;
        if (t == 0) xl[k] = xk;
        __syncthreads();
      }
    }
  } else {
    // one panel per step, last first; 8 lanes per panel row.  The panel's
    // A11^-1 is loaded into registers with the A12 rows, so that both loads
    // are in flight together, and applied from LDS.
    __shared__ double Ds[PANEL_NB][PANEL_NB + 1];
    static_assert(NT == 8 * PANEL_NB, "8 lanes per panel row");
    const int row = t / 8, lane = t % 8;
    const int np = (s + PANEL_NB - 1) / PANEL_NB;
    for (int p = np - 1; p >= 0; --p) {
      const int k0 = p * PANEL_NB, nb = min(PANEL_NB, s - k0);
      const double* Di = inv + nd.inv_off + (long long)p * PANEL_NB * PANEL_NB;
      double dreg[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) dreg[q] = Di[row * PANEL_NB + 4 * lane + q];
      // y = b_1 - A12 x_2, then a reduction across the row's lanes
      double v = 0.0;
      if (row < nb) {
        const double* fr = F + (long long)(k0 + row) * ld;
        const double bk = rv ? rv[k0 + row] : fr[n];   // in flight with the row's loads
        v = row_dot_sub<32>(v, fr, xl, k0 + nb + lane, n);
        if (lane == 0) v += bk;
      }
      for (int off = 4; off > 0; off >>= 1) v += __shfl_down(v, off, 8);
      if (row < nb && lane == 0) y[row] = v;
#pragma unroll
      for (int q = 0; q < 4; ++q) Ds[row][4 * lane + q] = dreg[q];
      __syncthreads();
      // x_1 = A11^-1 y: 4 products per lane, reduced across the row's lanes
      double u = 0.0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int m = 4 * lane + q;
        u += m < nb ? Ds[row][m] * y[m] : 0.0;
      }
      for (int off = 4; off > 0; off >>= 1) u += __shfl_down(u, off, 8);
      if (row < nb && lane == 0) xl[k0 + row] = u;
      __syncthreads();
    }
  }
  for (int k = t; k < s; k += NT) x[dof[k]] = xl[k];
}

// Forward elimination of a new right-hand side through one stored front:
// gather the children's eliminated rhs (extend-add with the same maps as
// the matrix), add the new values of the front's own separator dofs (each
// dof is eliminated at exactly one node, so each value enters once), and
// apply the stored elimination: multipliers in the columns of classic
// fronts; A21 A11^-1 per panel for blocked fronts (the panel rows keep their
// panel-time values for the back substitution).
__global__ void __launch_bounds__(NT) front_rhs_kernel(const NodeDesc* nodes, const double* tree,
                                                       const double* inv, const int2* maps,
                                                       const int* dofs, const double* r,
                                                       double* rtree) {
  extern __shared__ double rl[];   // n values
  __shared__ double z[PANEL_NB];
  const NodeDesc nd = nodes[blockIdx.x];
  const int n = nd.n, s = nd.s, ld = n + 1;
  const int t = threadIdx.x;
  const int2* mp = maps + nd.map_off;
  const int* dof = dofs + nd.dof_off;
  for (int a = t; a < n; a += NT) {
    const int2 ma = mp[a];
    double v = 0.0;
    if (ma.x >= 0 && nd.cr_off[0] >= 0) v += rtree[nd.cr_off[0] + ma.x];
    if (ma.y >= 0 && nd.cr_off[1] >= 0) v += rtree[nd.cr_off[1] + ma.y];
    if (a < s) v += r[dof[a]];
    rl[a] = v;
  }
  const double* F = tree + nd.f_off;
  if (!nd.blocked) {
    for (int k = 0; k < s; ++k) {
      __syncthreads();
      const double rk = rl[k];
      for (int a = k + 1 + t; a < n; a += NT) rl[a] -= F[(long long)a * ld + k] * rk;
    }
  } else {
    // per panel: z = A11^-1 y_panel, then y_a -= A_a,panel z for the rows
    // below; 8 lanes per row, 4 consecutive columns each (a row's 32 panel
    // entries are one 256-byte segment), reduced across the 8 lanes
    const int l8 = t & 7, row = t >> 3;   // 32 rows per pass
    for (int k0 = 0; k0 < s; k0 += PANEL_NB) {
      const int nb = min(PANEL_NB, s - k0);
      const double* Di = inv + nd.inv_off + (long long)(k0 / PANEL_NB) * PANEL_NB * PANEL_NB;
      __syncthreads();
      {
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int m = 4 * l8 + q;
          const bool in = row < nb && m < nb;
          const double d = Di[in ? row * PANEL_NB + m : 0];
          const double y = rl[in ? k0 + m : k0];
          v += in ? d * y : 0.0;
        }
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        if (row < nb && l8 == 0) z[row] = v;
      }
      __syncthreads();
      for (int a0 = k0 + nb; a0 < n; a0 += NT / 8) {
        const int a = a0 + row;
        const double* fr = F + (long long)(a < n ? a : k0 + nb) * ld + k0;
        double v = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int m = 4 * l8 + q;
          const double f = fr[m < nb ? m : 0];
          const double zm = z[m < nb ? m : 0];
          v += (a < n && m < nb) ? f * zm : 0.0;
        }
        v += __shfl_xor(v, 1);
        v += __shfl_xor(v, 2);
        v += __shfl_xor(v, 4);
        if (a < n && l8 == 0) rl[a] -= v;
      }
    }
  }
  __syncthreads();
  for (int a = t; a < n; a += NT) rtree[nd.r_off + a] = rl[a];
}

__global__ void add_kernel(double* x, const double* dx, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    x[i] += dx[i];
}

// r = b - A x gathered from the subdomain blocks (each interface row has
// two owners: its lower- and higher-index subdomain).  Stage 1: per
// work-group maxima of |r_i| and of the row's scale |b_i| + sum_j |A_ij x_j|
// (so that max |r| / max scale is a normwise backward error, which the
// rounding of an FP64 solve leaves near eps even where |A| |x| is far above
// |b|); stage 2: one work-group reduces them.
// interface edge on side (W, E, S, N) of subdomain (I, J), -1 on the
// domain boundary
__device__ inline int side_edge(const Geo& g, int I, int J, int side) {
  switch (side) {
    case 0: return I > 0 ? J * (g.SX - 1) + I - 1 : -1;
    case 1: return I < g.SX - 1 ? J * (g.SX - 1) + I : -1;
    case 2: return J > 0 ? g.nV + (J - 1) * g.SX + I : -1;
    default: return J < g.SY - 1 ? g.nV + J * g.SX + I : -1;
  }
}

// DT: the interface dofs per edge when fixed at compile time (all loads of a
// row issued together), 0 for any
template <int DT>
__global__ void __launch_bounds__(NT) iface_residual_kernel(Geo g, const double* blocks,
                                                            const double* x, double* rvec,
                                                            double* partials) {
  __shared__ double red[2][NT];
  const int D = DT > 0 ? DT : g.D, NBR = 4 * D, NBC = NBR + 1;
  const int n_iface = g.nV + g.SX * (g.SY - 1);
  const int ndof = n_iface * D;
  double rmax = 0.0, bmax = 0.0;
  for (int row = blockIdx.x * NT + threadIdx.x; row < ndof; row += gridDim.x * NT) {
    const int e = row / D, k = row % D;
    int sub[2], side[2];
    if (e < g.nV) {
      const int J = e / (g.SX - 1), I = e % (g.SX - 1);
      sub[0] = J * g.SX + I; side[0] = 1;
      sub[1] = sub[0] + 1; side[1] = 0;
    } else {
      const int h = e - g.nV;
      const int J = h / g.SX, I = h % g.SX;
      sub[0] = J * g.SX + I; side[0] = 3;
      sub[1] = sub[0] + g.SX; side[1] = 2;
    }
    double hi = 0.0, lo = 0.0, b = 0.0;   // residual b - A x in double-double
    double sabs = 0.0;                    // sum of |A_ij x_j| of the row
    if constexpr (DT > 0) {
      // all of the row's loads first, from clamped addresses (a side on the
      // domain boundary contributes the exact no-op 0 * 0), then the
      // accumulation in the order of the sides
      double bb[2], av[2][4][DT], xv[2][4][DT];
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        const int sd = sub[o];
        const int I = sd % g.SX, J = sd / g.SX;
        const double* blk = blocks + (size_t)sd * NBR * NBC + (size_t)(side[o] * D + k) * NBC;
        bb[o] = blk[NBR];
#pragma unroll
        for (int sd_side = 0; sd_side < 4; ++sd_side) {
          const int ee = side_edge(g, I, J, sd_side);
#pragma unroll
          for (int kk = 0; kk < DT; ++kk) {
            const double av_ = blk[sd_side * D + kk];
            const double xv_ = x[(size_t)max(ee, 0) * D + kk];
            av[o][sd_side][kk] = ee >= 0 ? av_ : 0.0;
            xv[o][sd_side][kk] = ee >= 0 ? xv_ : 0.0;
          }
        }
      }
#pragma unroll
      for (int o = 0; o < 2; ++o) {
        b += bb[o];
        two_sum(hi, lo, bb[o]);
#pragma unroll
        for (int sd_side = 0; sd_side < 4; ++sd_side)
#pragma unroll
          for (int kk = 0; kk < DT; ++kk) {
            two_prod_sub(hi, lo, av[o][sd_side][kk], xv[o][sd_side][kk]);
            sabs += fabs(av[o][sd_side][kk] * xv[o][sd_side][kk]);
          }
      }
    } else {
      for (int o = 0; o < 2; ++o) {
        const int sd = sub[o];
        const int I = sd % g.SX, J = sd / g.SX;
        const double* blk = blocks + (size_t)sd * NBR * NBC + (size_t)(side[o] * D + k) * NBC;
        b += blk[NBR];
        two_sum(hi, lo, blk[NBR]);
        for (int sd_side = 0; sd_side < 4; ++sd_side) {
          const int ee = side_edge(g, I, J, sd_side);
          if (ee < 0) continue;
          for (int kk = 0; kk < D; ++kk) {
            const double av = blk[sd_side * D + kk], xv = x[(size_t)ee * D + kk];
            two_prod_sub(hi, lo, av, xv);
            sabs += fabs(av * xv);
          }
        }
      }
    }
    const double res = hi + lo;
    if (rvec) rvec[row] = res;
    rmax = fmax(rmax, fabs(res));
    bmax = fmax(bmax, fabs(b) + sabs);
  }
  red[0][threadIdx.x] = rmax;
  red[1][threadIdx.x] = bmax;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    partials[2 * blockIdx.x] = red[0][0];
    partials[2 * blockIdx.x + 1] = red[1][0];
  }
}

__global__ void __launch_bounds__(NT) max_pairs_kernel(const double* partials, int count,
                                                       double* out2, unsigned long long* stamp) {
  __shared__ double red[2][NT];
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < count; i += NT) {
    a = fmax(a, partials[2 * i]);
    b = fmax(b, partials[2 * i + 1]);
  }
  red[0][threadIdx.x] = a;
  red[1][threadIdx.x] = b;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      red[0][threadIdx.x] = fmax(red[0][threadIdx.x], red[0][threadIdx.x + w]);
      red[1][threadIdx.x] = fmax(red[1][threadIdx.x], red[1][threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out2[0] = red[0][0];
    out2[1] = red[1][0];
    stamp_now(stamp);
  }
}

}  // namespace

hipError_t launch_front_small(const NodeDesc* nodes, int count, int max_n, double* tree,
                              const int2* maps, int* status, unsigned long long* stamp,
                              hipStream_t st) {
  // the smallest register tile that holds the level's largest front (the
  // plan keeps max_n <= SMALL_FRONT): rows TYN RI >= n, columns TXN CJ > n
  static_assert(TYN * 8 >= SMALL_FRONT && TXN * 3 > SMALL_FRONT, "register tile of the largest front");
#define SMALL_LAUNCH(RI, CJ) \
  hipLaunchKernelGGL((front_small_kernel<RI, CJ>), dim3(count), dim3(NT), 0, st, nodes, tree, maps, status, \
                     stamp)
  if (max_n <= 31) SMALL_LAUNCH(4, 1);
  else if (max_n <= 40) SMALL_LAUNCH(5, 2);
  else if (max_n <= 56) SMALL_LAUNCH(7, 2);
  else if (max_n <= 63) SMALL_LAUNCH(8, 2);
  else SMALL_LAUNCH(8, 3);
#undef SMALL_LAUNCH
  return hipGetLastError();
}

hipError_t launch_front_update(const NodeDesc* nodes, const PanelItem* items, int count, int k0,
                               double* tree, const int2* maps, double* inv, int* status,
                               unsigned long long* stamp, hipStream_t st) {
  if (k0 == 0)
    hipLaunchKernelGGL(front_update_kernel<true>, dim3(count), dim3(NT), 0, st, nodes, items, k0,
                       tree, maps, inv, status, stamp);
  else
    hipLaunchKernelGGL(front_update_kernel<false>, dim3(count), dim3(NT), 0, st, nodes, items, k0,
                       tree, maps, inv, status, stamp);
  return hipGetLastError();
}

hipError_t launch_front_back(const NodeDesc* nodes, int count, int max_n, const double* tree,
                             const double* inv, const int* dofs, const double* rtree, double* x,
                             hipStream_t st) {
  // LDS for the level's largest front (the plan guarantees n <= MAX_FRONT)
  const size_t lds = (size_t)max_n * sizeof(double);
  if (max_n > SMALL_FRONT)   // the plan's rule for a blocked level
    hipLaunchKernelGGL(front_back_kernel<true>, dim3(count), dim3(NT), lds, st, nodes, tree, inv, dofs,
                       rtree, x);
  else
    hipLaunchKernelGGL(front_back_kernel<false>, dim3(count), dim3(NT), lds, st, nodes, tree, inv, dofs,
                       rtree, x);
  return hipGetLastError();
}

hipError_t launch_front_rhs(const NodeDesc* nodes, int count, int max_n, const double* tree,
                            const double* inv, const int2* maps, const int* dofs, const double* r,
                            double* rtree, hipStream_t st) {
  hipLaunchKernelGGL(front_rhs_kernel, dim3(count), dim3(NT), (size_t)max_n * sizeof(double), st,
                     nodes, tree, inv, maps, dofs, r, rtree);
  return hipGetLastError();
}

hipError_t launch_add(double* x, const double* dx, int n, hipStream_t st) {
  hipLaunchKernelGGL(add_kernel, dim3(64), dim3(NT), 0, st, x, dx, n);
  return hipGetLastError();
}

hipError_t launch_iface_residual(const Geo& g, const double* blocks, const double* x, double* r,
                                 double* partials, double* out2, unsigned long long* stamp,
                                 hipStream_t st) {
  if (g.D == 4)
    hipLaunchKernelGGL(iface_residual_kernel<4>, dim3(RESID_WG), dim3(NT), 0, st, g, blocks, x, r,
                       partials);
  else if (g.D == 8)
    hipLaunchKernelGGL(iface_residual_kernel<8>, dim3(RESID_WG), dim3(NT), 0, st, g, blocks, x, r,
                       partials);
  else
    hipLaunchKernelGGL(iface_residual_kernel<0>, dim3(RESID_WG), dim3(NT), 0, st, g, blocks, x, r,
                       partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(max_pairs_kernel, dim3(1), dim3(NT), 0, st, partials, RESID_WG, out2, stamp);
  return hipGetLastError();
}

}  // namespace mrcm
