// Register-tile FP64 kernels for 32 x 32 subdomains with four interface
// dofs per side (the 2048 x 1024 workload), on the matrix cores of gfx950.
//
// The same method as the 16 x 16 kernels (paper, section 3: the local Robin
// problems of eq. (mrc1) and their basis functions, the traces projected on
// the interface spaces of eq. (mrc2); and the stitch re-solve), laid out for
// 32-cell block rows:
//
//  * A 32 x 32 Schur block is four 16 x 16 tiles in the FP64 MFMA output
//    layout (mfma_tile.h).  Its inverse is formed by blocks: the leading
//    tile P and the Schur complement C = B - Q^T P^{-1} Q are inverted by
//    register Gauss-Jordan sweeps, the off-diagonal blocks -P^{-1} Q C^{-1}
//    and the corrected leading block by matrix-core products, with one
//    transpose through LDS.
//  * Two wavefronts per subdomain eliminate the 32 block rows from both
//    ends (rows 0..15 downwards, rows 31..17 upwards) and meet at row 16.
//  * A chain's inverse blocks do not fit in registers (16 blocks of 16
//    doubles per lane): each is written once to the subdomain's scratch in
//    the lane layout (one 512-byte segment per register) and read back by
//    the backward sweep and by the refinement step.  The forward solution
//    of the basis columns goes to the output array and is overwritten by
//    the backward sweep.
//  * One step of iterative refinement with the double-double residual of
//    the cells' mass balances (exact diagonal), as in the 16 x 16 kernel.
#include "local_common.h"
#include "mfma_tile.h"

namespace mrcm {
namespace {

using namespace local;
using namespace tile;

constexpr int M = 32;
constexpr int MM = M * M;
constexpr int D = 4;
constexpr int R = 1 + 4 * D;
constexpr int PAIR = 128;
constexpr int JN = M / 2;   // joining block row

// per-subdomain scratch (doubles): inverse blocks, correction forward
// solutions, the hand-over at the join
constexpr long long SC_SINV = 0;                       // [row][16 regs][64 lanes]
constexpr long long SC_ZC = SC_SINV + (long long)M * 1024;   // [row][4 tiles][4][64]
constexpr long long SC_XCH = SC_ZC + (long long)M * 1024;    // block + 4 tiles
constexpr long long SC_RES = SC_XCH + 2048;                  // per wave: 4 tiles
constexpr long long SC_TOTAL = SC_RES + 2048;
// with windows of dofs (8 per side): each window's scratch, followed by its
// copy of the particular solution (SC_PART)
constexpr long long SC_PART = SC_TOTAL;
constexpr long long SC_WINDOW = SC_TOTAL + MM;

struct Blk {
  d4 t[2][2];   // tile (row block, column block)
};

// rows of a wavefront's chain: wave 0 owns rows 0..15, wave 1 rows 31..17
template <int W>
struct Chain32 {
  static constexpr int NR = W ? M - 1 - JN : JN;            // rows before the join
  static constexpr int row(int t) { return W ? M - 1 - t : t; }
  // coupling (row index of cy) to the previous row of the chain / towards the join
  static constexpr int cprev(int t) { return W ? M - 1 - t : t - 1; }
  static constexpr int cnext(int t) { return W ? M - 2 - t : t; }
};

__device__ __forceinline__ const d4 zero4() { return d4{0.0, 0.0, 0.0, 0.0}; }

// D_j - C P C (C = diag of coupling row jc; D_j alone when has_p is false)
__device__ __forceinline__ Blk coupled32(int j, int jc, const Blk& P, bool has_p, int c, int g,
                                         const double* dg, const double* ex, const double* cy) {
  Blk s;
  jc = jc < 0 ? 0 : jc;   // (no coupling row when has_p is false)
#pragma unroll
  for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
    for (int Cc = 0; Cc < 2; ++Cc)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * Rr + 4 * v + g, q = 16 * Cc + c;
        double d = (i == q) ? dg[j * M + i]
                 : (i == q + 1) ? ex[j * M + q]
                 : (q == i + 1) ? ex[j * M + i] : 0.0;
        if (has_p) d -= cy[jc * M + i] * P.t[Rr][Cc][v] * cy[jc * M + q];
        s.t[Rr][Cc][v] = d;
      }
  return s;
}

// In-place inverse of the symmetric positive definite block S by 2 x 2
// blocks; tr is the wavefront's 16 x 16 LDS tile for the transpose (element
// (r, q) at [r][q ^ r], which spreads a column over the banks).
__device__ __forceinline__ void invert32(Blk& S, double (*tr)[16], int c, int g, PivotCheck& pc) {
  const d4 z = zero4();
  const d4 Pi = gauss_jordan16(S.t[0][0], c, g, pc);
  const d4 X = mm_tn(Pi, S.t[0][1], z);                    // P^-1 Q
  const d4 Ci = gauss_jordan16(S.t[1][1] - mm_tn(S.t[0][1], X, z), c, g, pc);
#pragma unroll
  for (int v = 0; v < 4; ++v) tr[4 * v + g][c ^ (4 * v + g)] = X[v];
  __builtin_amdgcn_wave_barrier();
  d4 XT;
#pragma unroll
  for (int v = 0; v < 4; ++v) XT[v] = tr[c][(4 * v + g) ^ c];
  __builtin_amdgcn_wave_barrier();
  const d4 S10 = -mm_tn(Ci, XT, z);                        // -C^-1 X^T
  S.t[0][1] = -mm_tn(XT, Ci, z);                           // -X C^-1
  S.t[0][0] = Pi - mm_tn(S10, XT, z);                      // P^-1 + X C^-1 X^T
  S.t[1][0] = S10;
  S.t[1][1] = Ci;
}

// Si r for a right-hand side of two row tiles (tile (K, R) of the symmetric
// inverse, passed as the A operand, contributes its transpose (R, K))
__device__ __forceinline__ void apply_inv(const Blk& Si, const d4* r, d4* out) {
  const d4 z = zero4();
#pragma unroll
  for (int Rr = 0; Rr < 2; ++Rr) out[Rr] = mm_tn(Si.t[1][Rr], r[1], mm_tn(Si.t[0][Rr], r[0], z));
}

__device__ __forceinline__ void store_blk(double* dst, const Blk& b, int lane) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) dst[(4 * k + v) * 64 + lane] = b.t[k >> 1][k & 1][v];
}
__device__ __forceinline__ void load_blk(const double* src, Blk& b, int lane) {
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int v = 0; v < 4; ++v) b.t[k >> 1][k & 1][v] = src[(4 * k + v) * 64 + lane];
}
// four tiles (two row tiles of the basis columns, two of the particular)
__device__ __forceinline__ void store_t4(double* dst, const d4* zb, const d4* zp, int lane) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    dst[(0 + v) * 64 + lane] = zb[0][v];
    dst[(4 + v) * 64 + lane] = zb[1][v];
    dst[(8 + v) * 64 + lane] = zp[0][v];
    dst[(12 + v) * 64 + lane] = zp[1][v];
  }
}
__device__ __forceinline__ void load_t4(const double* src, d4* zb, d4* zp, int lane) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    zb[0][v] = src[(0 + v) * 64 + lane];
    zb[1][v] = src[(4 + v) * 64 + lane];
    zp[0][v] = src[(8 + v) * 64 + lane];
    zp[1][v] = src[(12 + v) * 64 + lane];
  }
}

// The refinement's forward solutions, kept in FP32 (they carry only the
// leading digits of corrections far below the solution, as in the 16 x 16
// kernel): half the scratch traffic of FP64 copies.  The particular
// column's tiles are the same in all 16 MFMA columns, so only the lanes of
// column 0 store them and every lane reads those.
__device__ __forceinline__ void store_t4f(float* dst, const d4* zb, const d4* zp, int lane) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    dst[(0 + v) * 64 + lane] = (float)zb[0][v];
    dst[(4 + v) * 64 + lane] = (float)zb[1][v];
  }
  if ((lane & 15) == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      dst[(8 + v) * 64 + lane] = (float)zp[0][v];
      dst[(12 + v) * 64 + lane] = (float)zp[1][v];
    }
  }
}
__device__ __forceinline__ void load_t4f(const float* src, d4* zb, d4* zp, int lane) {
  const int l0 = lane & 48;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    zb[0][v] = (double)src[(0 + v) * 64 + lane];
    zb[1][v] = (double)src[(4 + v) * 64 + lane];
    zp[0][v] = (double)src[(8 + v) * 64 + l0];
    zp[1][v] = (double)src[(12 + v) * 64 + l0];
  }
}

// right-hand side of basis column q (dof q of the W, E, S, N interfaces) at
// local cell (li, lj): non-zero next to the faces of its side only
__device__ __forceinline__ double side_rhs32(const double (*bside)[M][D], int lj, int li, int q) {
  const int side = q >> 2, k = q & 3;
  const bool on = side == 0 ? li == 0 : side == 1 ? li == M - 1 : side == 2 ? lj == 0 : lj == M - 1;
  const double v = bside[side][side < 2 ? lj : li][k];
  return on ? v : 0.0;
}

// Where a lane's columns live: colp(c), the basis column of lane column c;
// partp(), the particular solution.  XPlain: 4 dofs per side, the columns of
// X itself.  XWindow: one window of 4 dofs per side out of more (col, the
// lane's column of X); the particular solution is X's column 0 for the first
// window, and the other windows keep their own copy in their scratch, as
// only the first writes X's.
struct XPlain {
  double* x;
  __device__ double* colp(int c) const { return x + (size_t)(1 + c) * MM; }
  __device__ double* partp() const { return x; }
};
struct XWindow {
  double* x;
  int col;
  double* part;
  __device__ double* colp(int) const { return x + (size_t)col * MM; }
  __device__ double* partp() const { return part; }
};

// Solution tiles of row j: basis column c of the lane, the particular column
// replicated over the 16 MFMA columns, only the lanes of column 0 storing it.
template <class XV>
__device__ __forceinline__ void store_x(const XV& xv, int j, const d4* zb, const d4* zp, int c, int g) {
#pragma unroll
  for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int l = j * M + 16 * Rr + 4 * v + g;
      xv.colp(c)[l] = zb[Rr][v];
      if (c == 0) xv.partp()[l] = zp[Rr][v];
    }
}
template <class XV>
__device__ __forceinline__ void load_x(const XV& xv, int j, d4* zb, d4* zp, int c, int g) {
#pragma unroll
  for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int l = j * M + 16 * Rr + 4 * v + g;
      zb[Rr][v] = xv.colp(c)[l];
      zp[Rr][v] = xv.partp()[l];
    }
}

// LDS of the basis kernel
struct Lds32b {
  double kap[MM], dg[MM], ex[MM], cy[MM], b0[MM];
  float dgl[MM];              // rounding error of the diagonal sums
  double bside[4][M][D];      // Robin data of the basis columns per face
  double tr[2][16][16];       // per-wave transpose tiles
};

// Double-double residual of the cells' mass balances for the tiles of row j
// (basis column c and the particular column), from the solution in X.  The
// elements are formed two at a time into the lane's own slots of buf (the
// tile layout of store_t4) and read back as tiles: formed all together, their
// 96 operand loads would be in flight at once beside the inverse block (two
// at a time: 2% shorter than one at a time, with fewer spills; four or more
// spill more).
template <class XV>
__device__ __forceinline__ void residual_row(const Lds32b& sh, const XV& xv, int j, int c, int g,
                                             int lane, double* buf, d4* rb, d4* rp) {
#pragma unroll 2
  for (int e = 0; e < 16; ++e) {
    const int k = e >> 3, Rr = (e >> 2) & 1, v = e & 3;   // k: basis (0) or particular (1)
    const int i = 16 * Rr + 4 * v + g, l = j * M + i;
    // neighbour indices clamped (their coefficients are selected to 0)
    const int le = i < M - 1 ? l + 1 : l, lw = i > 0 ? l - 1 : l;
    const int ln = j < M - 1 ? l + M : l, ls = j > 0 ? l - M : l;
    const double ce = i < M - 1 ? sh.ex[l] : 0.0, cw = i > 0 ? sh.ex[lw] : 0.0;
    const double cn = j < M - 1 ? sh.cy[l] : 0.0, cs = j > 0 ? sh.cy[ls] : 0.0;
    const double* x = k == 0 ? xv.colp(c) : xv.partp();
    double hi = k == 0 ? side_rhs32(sh.bside, j, i, c) : sh.b0[l], lo = 0.0;
    const double xc = x[l];
    dd_fma(hi, lo, -sh.dg[l], xc);
    dd_fma_low(lo, -(double)sh.dgl[l], xc);
    dd_fma(hi, lo, -ce, x[le]);
    dd_fma(hi, lo, -cw, x[lw]);
    dd_fma(hi, lo, -cn, x[ln]);
    dd_fma(hi, lo, -cs, x[ls]);
    buf[(8 * k + 4 * Rr + v) * 64 + lane] = hi + lo;
  }
  load_t4(buf, rb, rp, lane);
}

// One wavefront's forward sweep.  FACTOR: form and invert the Schur blocks
// (written to scratch); else load them.  The right-hand side of row j comes
// from rhs(j, rb, rp); the forward solution goes to out(j, zb, zp).  Leaves
// the last row's inverse block and solution tiles in P, zb, zp.
template <int W, bool FACTOR, bool BASIS, class Rhs, class Out>
__device__ __forceinline__ void forward32(const double* dg, const double* ex, const double* cy,
                                          double (*tr)[16], double* scr, int c, int g, int lane,
                                          PivotCheck& pc, Blk& P, d4* zb, d4* zp, Rhs rhs, Out out) {
  using C = Chain32<W>;
#pragma unroll 1
  for (int t = 0; t < C::NR; ++t) {
    const int j = C::row(t);
    d4 rb[2], rp[2];
    rhs(j, rb, rp);
    if (FACTOR) {
      Blk S = coupled32(j, C::cprev(t), P, t > 0, c, g, dg, ex, cy);
      invert32(S, tr, c, g, pc);
      store_blk(scr + SC_SINV + (long long)j * 1024, S, lane);
      P = S;
    } else {
      load_blk(scr + SC_SINV + (long long)j * 1024, P, lane);
    }
    if (t > 0) {
      const int jc = C::cprev(t);
#pragma unroll
      for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const double cc = cy[jc * M + 16 * Rr + 4 * v + g];
          if (BASIS) rb[Rr][v] -= cc * zb[Rr][v];
          rp[Rr][v] -= cc * zp[Rr][v];
        }
    }
    if (BASIS) apply_inv(P, rb, zb);
    apply_inv(P, rp, zp);
    out(j, zb, zp);
  }
}

// The joining row (wave 0): its Schur block from both chains' last inverse
// blocks, and its solution, which is final.  Pn, zbn, zpn: wave 1's row 17.
template <bool FACTOR, bool BASIS, class Rhs>
__device__ __forceinline__ void join32(const double* dg, const double* ex, const double* cy,
                                       double (*tr)[16], double* scr, int c, int g, int lane,
                                       PivotCheck& pc, const Blk& P, const d4* zb, const d4* zp,
                                       const Blk& Pn, const d4* zbn, const d4* zpn, d4* xb, d4* xp,
                                       Rhs rhs) {
  constexpr int j = JN;
  Blk S;
  if (FACTOR) {
    S = coupled32(j, j - 1, P, true, c, g, dg, ex, cy);
#pragma unroll
    for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
      for (int Cc = 0; Cc < 2; ++Cc)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 16 * Rr + 4 * v + g, q = 16 * Cc + c;
          S.t[Rr][Cc][v] -= cy[j * M + i] * Pn.t[Rr][Cc][v] * cy[j * M + q];
        }
    invert32(S, tr, c, g, pc);
    store_blk(scr + SC_SINV + (long long)j * 1024, S, lane);
  } else {
    load_blk(scr + SC_SINV + (long long)j * 1024, S, lane);
  }
  d4 rb[2], rp[2];
  rhs(j, rb, rp);
#pragma unroll
  for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 16 * Rr + 4 * v + g;
      const double cu = cy[(j - 1) * M + i], cd = cy[j * M + i];
      if (BASIS) rb[Rr][v] -= cu * zb[Rr][v] + cd * zbn[Rr][v];
      rp[Rr][v] -= cu * zp[Rr][v] + cd * zpn[Rr][v];
    }
  if (BASIS) apply_inv(S, rb, xb);
  apply_inv(S, rp, xp);
}

// One wavefront's backward sweep from the join: x_j = z_j - Si_j C x_next;
// z(j, zb, zp) gives the forward solution of row j, put(j, xb, xp) takes x_j.
template <int W, bool BASIS, class Z, class Put>
__device__ __forceinline__ void backward32(const double* cy, const double* scr, int c, int g, int lane,
                                           const d4* xb_join, const d4* xp_join, Z z, Put put) {
  using C = Chain32<W>;
  d4 xb[2] = {xb_join[0], xb_join[1]}, xp[2] = {xp_join[0], xp_join[1]};
#pragma unroll 1
  for (int t = C::NR - 1; t >= 0; --t) {
    const int j = C::row(t), jc = C::cnext(t);
    Blk Si;
    load_blk(scr + SC_SINV + (long long)j * 1024, Si, lane);
    d4 tb[2], tp[2];
#pragma unroll
    for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double cc = -cy[jc * M + 16 * Rr + 4 * v + g];
        if (BASIS) tb[Rr][v] = cc * xb[Rr][v];
        tp[Rr][v] = cc * xp[Rr][v];
      }
    d4 zb[2], zp[2], ub[2], up[2];
    z(j, zb, zp);
    if (BASIS) apply_inv(Si, tb, ub);
    apply_inv(Si, tp, up);
#pragma unroll
    for (int Rr = 0; Rr < 2; ++Rr) {
      if (BASIS) xb[Rr] = zb[Rr] + ub[Rr];
      xp[Rr] = zp[Rr] + up[Rr];
    }
    put(j, xb, xp);
  }
}

// Robin data of the basis columns of one window of 4 dofs per side (dofs
// 4 win .. 4 win + 3 of DD) per skeleton face: T_R g_k(t), with the flux
// functions scaled by -beta sigma (zero on the domain boundary)
template <int DD>
__device__ __forceinline__ void robin_data32(const SubArgs& a, int I, int J, const double* kap,
                                    double (*bside)[M][D], int win) {
  const Geo& g = a.g;
  for (int o = threadIdx.x; o < 4 * M; o += blockDim.x) {
    const int side = o / M, t = o % M;
    const int e = side_iface(g, I, J, side);
    double v[D] = {0.0, 0.0, 0.0, 0.0};
    if (e >= 0) {
      const SideGeo sg = side_geo(g, side);
      const double al = a.alpha[e];
      const double kk = kap[side_cell<M>(side, t)];
      const double TR = sg.flen * kk / (sg.dist + al * sg.H);
      const double beta = al * sg.H / kk;
      const double sig = side_sigma(side);
      const double* bs = a.basis + (size_t)e * DD * M;
#pragma unroll
      for (int k = 0; k < D; ++k) {
        const int kg = 4 * win + k;
        const double ph = bs[kg * M + t];
        v[k] = TR * (kg < g.nP ? ph : -beta * sig * ph);
      }
    }
#pragma unroll
    for (int k = 0; k < D; ++k) bside[side][t][k] = v[k];
  }
}

template <int W, class XV>
__device__ __forceinline__ void basis32_wave(const SubArgs& a, Lds32b& sh, int sd, double* scr, const XV& xv) {
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  PivotCheck pc;
  Blk P;
  d4 zb[2], zp[2];
  auto rhs_b = [&](int j, d4* rb, d4* rp) {
#pragma unroll
    for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 16 * Rr + 4 * v + g;
        rb[Rr][v] = side_rhs32(sh.bside, j, i, c);
        rp[Rr][v] = sh.b0[j * M + i];
      }
  };
  auto out_x = [&](int j, const d4* b, const d4* p) { store_x(xv, j, b, p, c, g); };
  // factorisation and forward solve; the join; backward solve
  forward32<W, true, true>(sh.dg, sh.ex, sh.cy, sh.tr[W], scr, c, g, lane, pc, P, zb, zp, rhs_b, out_x);
  double* xch = scr + SC_XCH;
  if (W == 1) {
    store_blk(xch, P, lane);
    store_t4(xch + 1024, zb, zp, lane);
  }
  __syncthreads();
  d4 xb[2], xp[2];
  if (W == 0) {
    Blk Pn;
    d4 zbn[2], zpn[2];
    load_blk(xch, Pn, lane);
    load_t4(xch + 1024, zbn, zpn, lane);
    join32<true, true>(sh.dg, sh.ex, sh.cy, sh.tr[0], scr, c, g, lane, pc, P, zb, zp, Pn, zbn, zpn, xb, xp,
                       rhs_b);
    store_x(xv, JN, xb, xp, c, g);
  }
  __syncthreads();
  if (W == 0) store_t4(xch + 1024, xb, xp, lane);   // the join's solution for wave 1
  __syncthreads();
  if (W == 1) load_t4(xch + 1024, xb, xp, lane);
  auto z_x = [&](int j, d4* b, d4* p) { load_x(xv, j, b, p, c, g); };
  backward32<W, true>(sh.cy, scr, c, g, lane, xb, xp, z_x, out_x);
  if (pc.bad()) atomicOr(a.status, ST_LOCAL_PIVOT);
  __syncthreads();

  // one refinement step: the residual of each row is formed just before the
  // row's correction is eliminated (the solution in X is final there); the
  // correction's forward solution goes to scratch, the backward sweep adds
  // the correction to X
  double* zc = scr + SC_ZC;
  double* rbuf = scr + SC_RES + (long long)W * 1024;   // the wave's residual slots
  auto rhs_r = [&](int j, d4* rb, d4* rp) { residual_row(sh, xv, j, c, g, lane, rbuf, rb, rp); };
  float* zcf = reinterpret_cast<float*>(zc);
  auto out_zc = [&](int j, const d4* b, const d4* p) { store_t4f(zcf + (long long)j * 1024, b, p, lane); };
  forward32<W, false, true>(sh.dg, sh.ex, sh.cy, sh.tr[W], scr, c, g, lane, pc, P, zb, zp, rhs_r, out_zc);
  __syncthreads();   // every residual is formed before any correction is added
  if (W == 1) store_t4(xch + 1024, zb, zp, lane);
  __syncthreads();
  if (W == 0) {
    Blk Pn;
    d4 zbn[2], zpn[2];
    load_t4(xch + 1024, zbn, zpn, lane);
    join32<false, true>(sh.dg, sh.ex, sh.cy, sh.tr[0], scr, c, g, lane, pc, P, zb, zp, Pn, zbn, zpn, xb, xp,
                        rhs_r);
  }
  __syncthreads();
  if (W == 0) store_t4(xch + 1024, xb, xp, lane);
  __syncthreads();
  if (W == 1) load_t4(xch + 1024, xb, xp, lane);
  auto add_x = [&](int j, const d4* b, const d4* p) {
    d4 ob[2], op[2];
    load_x(xv, j, ob, op, c, g);
    d4 nb[2] = {ob[0] + b[0], ob[1] + b[1]}, np[2] = {op[0] + p[0], op[1] + p[1]};
    store_x(xv, j, nb, np, c, g);
  };
  if (W == 0) add_x(JN, xb, xp);
  auto z_c = [&](int j, d4* b, d4* p) { load_t4f(zcf + (long long)j * 1024, b, p, lane); };
  backward32<W, true>(sh.cy, scr, c, g, lane, xb, xp, z_c, add_x);
}

// FP64 basis functions of 32 x 32 subdomains (LIST: only the subdomains on
// the fallback list of the FP32 kernel).  Two wavefronts per subdomain; with
// DD = 8 dofs per side, DD / 4 windows of 4 dofs per side, one work-group
// each (work-group b: subdomain b / (DD / 4), window b % (DD / 4), its own
// scratch), every window factorising the subdomain's matrix.  With 4 dofs
// per side, one wavefront per SIMD: the 25 dwords per lane that spilled to
// scratch at two stay in accumulation registers (the launch about 3% shorter
// at 2048 x 1024); with 8, two wavefronts per SIMD measured faster.
template <bool LIST, int DD>
__global__ void __launch_bounds__(PAIR, DD == 4 ? 1 : 2) basis32x32_kernel(SubArgs a) {
  static_assert(DD % 4 == 0 && (!LIST || DD == 4), "windows of 4 dofs per side");
  constexpr int NW = DD / 4, RX = 4 * DD + 1;
  __shared__ Lds32b sh;
  const Geo& g = a.g;
  int sd = NW == 1 ? (int)blockIdx.x : (int)blockIdx.x / NW;
  const int win = NW == 1 ? 0 : (int)blockIdx.x % NW;
  if (LIST) {
    if ((int)blockIdx.x >= a.fallback[0]) return;
    sd = a.fallback[1 + blockIdx.x];
  }
  const int I = sd % g.SX, J = sd / g.SX;
  const int tid = threadIdx.x, c = tid & 15;
  double* scr = a.scratch + (size_t)sd * a.scratch_stride + (size_t)win * SC_WINDOW;
  double* Xg = a.X + (size_t)sd * RX * MM;
  load_kappa<M>(a, I, J, sh.kap);
  __syncthreads();
  for (int l = tid; l < MM; l += PAIR)
    assemble_cell<M, 1, false>(a, I, J, l, sh.kap, sh.dg, sh.ex, sh.cy, sh.b0 + l, 1, nullptr, sh.dgl);
  robin_data32<DD>(a, I, J, sh.kap, sh.bside, win);
  __syncthreads();
  if constexpr (NW == 1) {
    const XPlain xv{Xg};
    if (__builtin_amdgcn_readfirstlane(tid >> 6) == 0) basis32_wave<0>(a, sh, sd, scr, xv);
    else basis32_wave<1>(a, sh, sd, scr, xv);
  } else {
    const XWindow xv{Xg, 1 + (c >> 2) * DD + 4 * win + (c & 3), win == 0 ? Xg : scr + SC_PART};
    if (__builtin_amdgcn_readfirstlane(tid >> 6) == 0) basis32_wave<0>(a, sh, sd, scr, xv);
    else basis32_wave<1>(a, sh, sd, scr, xv);
  }
  __syncthreads();
  generic_block<M, DD>(a, sd, I, J, sh.kap, Xg, 1, MM, NW == 1 ? -1 : win);
}

// ---------------------------------------------------------------------------
// stitch re-solve for 32 x 32 subdomains (two wavefronts per subdomain)
// ---------------------------------------------------------------------------

// scratch areas of the stitch (doubles): the inverse blocks at SC_SINV, the
// correction's forward solution (two tiles per row), the first solution ps,
// its residual rs and correction pl (cell-indexed), the join hand-over
constexpr long long SS_ZC = SC_SINV + (long long)M * 1024;
constexpr long long SS_PS = SS_ZC + (long long)M * 512;
constexpr long long SS_RS = SS_PS + MM;
constexpr long long SS_PL = SS_RS + MM;
constexpr long long SS_XCH = SS_PL + MM;
constexpr long long SS_TOTAL = SS_XCH + 2048;

template <int DD>
struct Lds32s {
  double kap[MM], dg[MM], ex[MM], cy[MM], pm[MM], bs[MM];
  double Fout[4][M];          // outflow of this subdomain on its skeleton faces
  double tr[2][16][16];       // per-wave transpose tiles
  double cfs[4 * DD];         // interface coefficients of the basis columns
  double red[2][2];
  double pin[2];              // per-cell defect share, pin transmissibility
};

__device__ __forceinline__ void store_t2(double* dst, const d4* zp, int lane) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    dst[v * 64 + lane] = zp[0][v];
    dst[(4 + v) * 64 + lane] = zp[1][v];
  }
}
__device__ __forceinline__ void load_t2(const double* src, d4* zp, int lane) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    zp[0][v] = src[v * 64 + lane];
    zp[1][v] = src[(4 + v) * 64 + lane];
  }
}

// composed pressure p = X [1; coefficients] at cell l of subdomain sd (4 DD
// basis columns; the loads issued 16 at a time)
template <int DD>
__device__ __forceinline__ double compose32(const SubArgs& a, int sd, int l, const double* cf) {
  const double* xr = a.X + (size_t)sd * (4 * DD + 1) * MM + l;
  if constexpr (DD == 4) {
    double x[4 * DD];
#pragma unroll
    for (int q = 0; q < 4 * DD; ++q) x[q] = xr[(size_t)(1 + q) * MM];
    double p = xr[0];
#pragma unroll
    for (int q = 0; q < 4 * DD; ++q) p = fma(x[q], cf[q], p);
    return p;
  } else {
    double p = xr[0];
#pragma unroll
    for (int q0 = 0; q0 < 4 * DD; q0 += 16) {
      double x[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) x[q] = xr[(size_t)(1 + q0 + q) * MM];
#pragma unroll
      for (int q = 0; q < 16; ++q) p = fma(x[q], cf[q0 + q], p);
    }
    return p;
  }
}

// One wavefront's solve of the stitch system for one column (rhs(j, rp)
// fills the tiles of row j, replicated over the 16 MFMA columns) into the
// cell array dst; FACTOR: form and store the inverse blocks first.
template <int W, bool FACTOR, class Rhs, class Sh>
__device__ __forceinline__ void stitch_solve32(Sh& sh, double* scr, int c, int g, int lane,
                                               PivotCheck& pc, double* dst, Rhs rhs) {
  Blk P;
  d4 zb[2], zp[2];
  auto rhs2 = [&](int j, d4* rb, d4* rp) { rhs(j, rp); };
  double* zc = scr + SS_ZC;
  auto keep = [&](int j, const d4* b, const d4* p) { store_t2(zc + (long long)j * 512, p, lane); };
  forward32<W, FACTOR, false>(sh.dg, sh.ex, sh.cy, sh.tr[W], scr, c, g, lane, pc, P, zb, zp, rhs2, keep);
  double* xch = scr + SS_XCH;
  if (W == 1) {
    if (FACTOR) store_blk(xch, P, lane);
    store_t2(xch + 1024, zp, lane);
  }
  __syncthreads();
  d4 xb[2], xp[2];
  if (W == 0) {
    Blk Pn;
    d4 zpn[2];
    if (FACTOR) load_blk(xch, Pn, lane);
    load_t2(xch + 1024, zpn, lane);
    join32<FACTOR, false>(sh.dg, sh.ex, sh.cy, sh.tr[0], scr, c, g, lane, pc, P, zb, zp, Pn, zb, zpn,
                          xb, xp, rhs2);
  }
  __syncthreads();
  if (W == 0) store_t2(xch + 1024, xp, lane);
  __syncthreads();
  if (W == 1) load_t2(xch + 1024, xp, lane);
  auto put = [&](int j, const d4* b, const d4* p) {
    if (c == 0) {
#pragma unroll
      for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
        for (int v = 0; v < 4; ++v) dst[j * M + 16 * Rr + 4 * v + g] = p[Rr][v];
    }
  };
  if (W == 0) put(JN, xb, xp);
  auto z = [&](int j, d4* b, d4* p) { load_t2(zc + (long long)j * 512, p, lane); };
  backward32<W, false>(sh.cy, scr, c, g, lane, xb, xp, z, put);
}

template <int W, class Sh>
__device__ __forceinline__ void stitch32_wave(const SubArgs& a, Sh& sh, double* scr, int I, int J) {
  const int lane = threadIdx.x & 63, c = lane & 15, g = lane >> 4;
  PivotCheck pc;
  double* ps = scr + SS_PS;
  double* rs = scr + SS_RS;
  double* pl = scr + SS_PL;
  auto rhs_b = [&](int j, d4* rp) {
#pragma unroll
    for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
      for (int v = 0; v < 4; ++v) rp[Rr][v] = sh.bs[j * M + 16 * Rr + 4 * v + g];
  };
  stitch_solve32<W, true>(sh, scr, c, g, lane, pc, ps, rhs_b);
  if (pc.bad()) atomicOr(a.status, ST_STITCH_PIVOT);
  __syncthreads();
  // residual of the cells' mass balances (double-double), then the
  // correction solve with the stored inverse blocks; the pressure is kept
  // as the unevaluated sum ps + pl, from which the fluxes are formed
  for (int l = threadIdx.x; l < MM; l += PAIR)
    rs[l] = stitch_balance_residual<M>(a, I, J, l, sh.kap, ps, sh.Fout, sh.pin[0], sh.pin[1], sh.pm[0]);
  __syncthreads();
  auto rhs_r = [&](int j, d4* rp) {
#pragma unroll
    for (int Rr = 0; Rr < 2; ++Rr)
#pragma unroll
      for (int v = 0; v < 4; ++v) rp[Rr][v] = rs[j * M + 16 * Rr + 4 * v + g];
  };
  stitch_solve32<W, false>(sh, scr, c, g, lane, pc, pl, rhs_r);
}

template <int DD>
__global__ void __launch_bounds__(PAIR, 2) stitch32x32_kernel(SubArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) stamp_now(a.stamps + STAMP_FLUX);
  __shared__ Lds32s<DD> sh;
  const Geo& g = a.g;
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int sd = blockIdx.x, I = sd % g.SX, J = sd / g.SX;
  double* scr = a.scratch + (size_t)sd * a.scratch_stride;
  if (tid < 4 * DD) {
    const int e = side_iface(g, I, J, tid / DD);
    sh.cfs[tid] = e >= 0 ? a.coef[(size_t)e * DD + tid % DD] : 0.0;
  }
  load_kappa<M>(a, I, J, sh.kap);
  __syncthreads();
  for (int l = tid; l < MM; l += PAIR) sh.pm[l] = compose32<DD>(a, sd, l, sh.cfs);
  __syncthreads();
  // one-sided Robin fluxes on both sides of each skeleton face, and their
  // average (the outflow of this subdomain)
  for (int o = tid; o < 4 * M; o += PAIR) {
    const int side = o / M, t = o % M;
    const int e = side_iface(g, I, J, side);
    double fo = 0.0;
    if (e >= 0) {
      const SideGeo sg = side_geo(g, side);
      const double al = a.alpha[e];
      const double* bsf = a.basis + (size_t)e * DD * M;
      const double* ce = a.coef + (size_t)e * DD;
      double PH = 0.0, UH = 0.0;
      for (int k = 0; k < g.nP; ++k) PH += ce[k] * bsf[k * M + t];
      for (int k = g.nP; k < DD; ++k) UH += ce[k] * bsf[k * M + t];
      const int l = side_cell<M>(side, t);
      const double sig = side_sigma(side);
      const double ko = sh.kap[l];
      const double TRo = sg.flen * ko / (sg.dist + al * sg.H);
      const double Fown = TRo * (sh.pm[l] - (PH - al * sg.H / ko * sig * UH)) +
                          robin_grav(a, side, (size_t)(J * M + l / M) * g.nx + I * M + l % M, TRo, sg.dist);
      const int nsd = (side == 0) ? sd - 1 : (side == 1) ? sd + 1 : (side == 2) ? sd - g.SX : sd + g.SX;
      const int nI = nsd % g.SX, nJ = nsd / g.SX;
      const int nl = side_cell<M>(side ^ 1, t);
      const size_t nc = (size_t)(nJ * M + nl / M) * g.nx + nI * M + nl % M;
      const double kn = a.K[nc] * a.lam[nc];
      double cfn[4 * DD];
#pragma unroll
      for (int q = 0; q < 4 * DD; ++q) {
        const int en = side_iface(g, nI, nJ, q / DD);
        cfn[q] = en >= 0 ? a.coef[(size_t)en * DD + q % DD] : 0.0;
      }
      const double pn = compose32<DD>(a, nsd, nl, cfn);
      const double TRn = sg.flen * kn / (sg.dist + al * sg.H);
      const double Fnb = TRn * (pn - (PH - al * sg.H / kn * (-sig) * UH)) + robin_grav(a, side ^ 1, nc, TRn, sg.dist);
      fo = 0.5 * (Fown - Fnb);
    }
    sh.Fout[side][t] = fo;
  }
  __syncthreads();
  for (int l = tid; l < MM; l += PAIR)
    assemble_cell<M, 1>(a, I, J, l, sh.kap, sh.dg, sh.ex, sh.cy, sh.bs + l, 0, sh.Fout);
  __syncthreads();
  // a subdomain with no Dirichlet face: the Neumann data's compatibility
  // defect (double-double sum) removed evenly from its cells, and the
  // constant fixed at cell 0 to the composed pressure
  const bool dir = (I == 0 && g.kind[0] == 1) || (I == g.SX - 1 && g.kind[1] == 1) ||
                   (J == 0 && g.kind[2] == 1) || (J == g.SY - 1 && g.kind[3] == 1);
  if (tid == 0) {
    sh.pin[0] = 0.0;
    sh.pin[1] = 0.0;
  }
  if (!dir) {
    double hs = 0.0, ls = 0.0;
    for (int l = tid; l < MM; l += PAIR) dd_add(hs, ls, sh.bs[l]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double oh = __shfl_xor(hs, off), ol = __shfl_xor(ls, off);
      dd_add(hs, ls, oh);
      ls += ol;
    }
    if (lane == 0) {
      sh.red[0][w] = hs;
      sh.red[1][w] = ls;
    }
    __syncthreads();
    hs = sh.red[0][0];
    ls = sh.red[1][0];
    dd_add(hs, ls, sh.red[0][1]);
    ls += sh.red[1][1];
    const double dfc = (hs + ls) / MM;
    for (int l = tid; l < MM; l += PAIR) sh.bs[l] -= dfc;
    if (tid == 0) {   // thread 0 owns cell 0
      const double tp = sh.dg[0];
      sh.dg[0] += tp;
      sh.bs[0] += tp * sh.pm[0];
      sh.pin[0] = dfc;
      sh.pin[1] = tp;
    }
  }
  __syncthreads();
  if (w == 0) stitch32_wave<0>(a, sh, scr, I, J);
  else stitch32_wave<1>(a, sh, scr, I, J);
  __syncthreads();

  const double* ps = scr + SS_PS;
  const double* pl = scr + SS_PL;
  double imb = 0.0, fmx = 0.0, psum = 0.0;
  for (int l = tid; l < MM; l += PAIR) {
    const int li = l % M, lj = l / M;
    const int i = I * M + li, j = J * M + lj;
    double out[4];
    stitch_out_fluxes<M>(a, I, J, l, sh.kap, ps, pl, sh.Fout, out);
    double F[4];
#pragma unroll
    for (int side = 0; side < 4; ++side) F[side] = (side == 0 || side == 2) ? -out[side] : out[side];
    a.ux[(size_t)j * (g.nx + 1) + i] = F[0] / g.hy;
    if (li == M - 1 && I == g.SX - 1) a.ux[(size_t)j * (g.nx + 1) + i + 1] = F[1] / g.hy;
    a.uy[(size_t)j * g.nx + i] = F[2] / g.hx;
    if (lj == M - 1 && J == g.SY - 1) a.uy[(size_t)(j + 1) * g.nx + i] = F[3] / g.hx;
    const double q = a.src ? a.src[(size_t)j * g.nx + i] * g.hx * g.hy : 0.0;
    const double net = F[1] - F[0] + F[3] - F[2];
    imb = fmax(imb, fabs(net - q));
    fmx = fmax(fmx, fmax(fmax(fabs(F[0]), fabs(F[1])), fmax(fabs(F[2]), fabs(F[3]))));
    a.p_out[(size_t)j * g.nx + i] = sh.pm[l];
    psum += sh.pm[l];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    imb = fmax(imb, __shfl_xor(imb, off));
    fmx = fmax(fmx, __shfl_xor(fmx, off));
    psum += __shfl_xor(psum, off);
  }
  __syncthreads();
  if (lane == 0) {
    sh.red[0][w] = imb;
    sh.red[1][w] = fmx;
    sh.pin[w] = psum;
  }
  __syncthreads();
  if (tid == 0) {
    a.sub_stats[3 * sd + 0] = fmax(sh.red[0][0], sh.red[0][1]);
    a.sub_stats[3 * sd + 1] = fmax(sh.red[1][0], sh.red[1][1]);
    a.sub_stats[3 * sd + 2] = sh.pin[0] + sh.pin[1];
  }
}

}  // namespace

bool basis32x32_supported(const Geo& g) {
  return g.M == M && !g.generic && ((g.D == 4 && g.nP == 2) || (g.D == 8 && g.prec == 0));
}

long long basis32x32_scratch(const Geo& g) {
  const long long basis = g.D == 4 ? SC_TOTAL : (g.D / 4) * SC_WINDOW;   // one scratch per window
  return basis > SS_TOTAL ? basis : SS_TOTAL;
}

hipError_t launch_stitch32x32(const SubArgs& a, hipStream_t st) {
  if (a.scratch_stride < SS_TOTAL) return hipErrorInvalidValue;
  if (a.g.D == 8)
    hipLaunchKernelGGL(stitch32x32_kernel<8>, dim3(a.g.n_sub), dim3(PAIR), 0, st, a);
  else
    hipLaunchKernelGGL(stitch32x32_kernel<4>, dim3(a.g.n_sub), dim3(PAIR), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_basis32x32(const SubArgs& a, hipStream_t st, bool list) {
  if (a.scratch_stride < basis32x32_scratch(a.g)) return hipErrorInvalidValue;
  if (a.g.D == 8) {
    if (list) return hipErrorInvalidValue;   // no FP32 form with 8 dofs per side
    hipLaunchKernelGGL((basis32x32_kernel<false, 8>), dim3(2 * a.g.n_sub), dim3(PAIR), 0, st, a);
  } else if (list) {
    hipLaunchKernelGGL((basis32x32_kernel<true, 4>), dim3(a.g.n_sub), dim3(PAIR), 0, st, a);
  } else {
    hipLaunchKernelGGL((basis32x32_kernel<false, 4>), dim3(a.g.n_sub), dim3(PAIR), 0, st, a);
  }
  return hipGetLastError();
}

}  // namespace mrcm
