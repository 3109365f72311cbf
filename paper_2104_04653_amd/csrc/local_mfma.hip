// Register-tile kernels for 16 x 16 subdomains with two pressure and two
// flux functions per interface (gfx950, FP64 MFMA).
//
// Same method as the generic kernels in local.hip (paper, section 3: local
// Robin problems of eq. (mrc1), basis functions, traces projected on the
// interface spaces of eq. (mrc2); and the stitch re-solve), laid out for the
// matrix cores:
//
//  * Every 16 x 16 tile is held in the output layout of
//    v_mfma_f64_16x16x4f64: lane l = c + 16 g (c = l & 15, g = l >> 4) holds
//    rows g, g+4, g+8, g+12 of column c in its four registers (row 4v + g in
//    register v).
//  * Block row j of the local matrix is inverted by Gauss-Jordan sweeps on
//    that register tile; the pivot row, pivot column and pivot element are
//    broadcast with lane shuffles, so no work-group barrier is needed.
//  * The products S_j^{-1} R and S_j^{-1} (C_j X_{j+1}) run on the matrix
//    cores.  The K index of the four K=4 steps is assigned as k = 4 kk + g
//    (step kk, lane group g), so the B operand of step kk is element kk of
//    the lane's own output-layout registers and the A operand is element kk
//    of the (symmetric) inverse in the same layout: no data moves between
//    lanes.  The 16 basis columns fill one MFMA tile; the particular
//    solution is a second tile with the right-hand side replicated over its
//    16 columns.
//  * Two-sided ("twisted") block elimination: one chain eliminates block
//    rows 0 .. MID-1 downwards, the other rows M-1 .. MID+1 upwards, and
//    block row MID joins them, which shortens the dependent chain of
//    Schur-block inversions from 16 to 9.  The FP64 basis and stitch kernels
//    give each chain its own wavefront; the inverse blocks and solution
//    tiles of a chain stay in that wavefront's registers for the backward
//    sweep.
#include "local_common.h"
#include "mfma_tile.h"

namespace mrcm {

namespace {

using namespace local;
using namespace tile;

typedef float f4z __attribute__((ext_vector_type(4)));

// the forward sweep of a refinement correction is kept in FP32 registers:
// it only carries the few leading digits of a correction that is itself
// orders of magnitude below the solution
__device__ inline f4z tof(d4 x) { return f4z{(float)x[0], (float)x[1], (float)x[2], (float)x[3]}; }
__device__ inline d4 tod(f4z x) { return d4{(double)x[0], (double)x[1], (double)x[2], (double)x[3]}; }

constexpr int M = 16;
constexpr int MM = 256;
constexpr int D = 4;
constexpr int R = 17;
constexpr int WAVE = 64;
constexpr int MID = M / 2;   // joining block row of the two-sided elimination

// D_j - C P C with C = diag(cy of coupling row jc) in output layout (D_j
// alone for jc < 0): the Schur-complemented diagonal block of row j after
// eliminating the neighbouring row whose inverse block is P.
__device__ inline d4 coupled_block(int j, int jc, const d4& P, int c, int g, const double* dg,
                                   const double* ex, const double* cy) {
  d4 s;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 4 * v + g;
    double d = (row == c) ? dg[j * M + row]
             : (row == c + 1) ? ex[j * M + c]
             : (c == row + 1) ? ex[j * M + row] : 0.0;
    if (jc >= 0) d -= cy[jc * M + row] * P[v] * cy[jc * M + c];
    s[v] = d;
  }
  return s;
}

// right-hand side of basis column c (dof c of the W, E, S, N interfaces) at
// local cell (li, lj): non-zero only next to the face of its side
__device__ inline double side_rhs(const double (*bside)[M][D], int lj, int li, int c) {
  const int side = c >> 2, k = c & 3;
  const bool on = side == 0 ? li == 0 : side == 1 ? li == M - 1 : side == 2 ? lj == 0 : lj == M - 1;
  const double v = bside[side][side < 2 ? lj : li][k];
  return on ? v : 0.0;
}

// Per skeleton face (side, t) of a subdomain: Robin transmissibility T_R,
// beta = alpha H / kappa and beta / |f| (all 0 on the domain boundary), and
// the DD interface functions of the side.  Computed once per kernel by the
// first 4 M threads; used by the Robin right-hand sides and by write_block.
template <int DD>
struct FacesT {
  double tr[4][M], bt[4][M], bl[4][M];
  double phi[4][DD][M];
  double gr[4][M];   // gravity part of the particular solution's Robin flux (0 without gravity)
};
using Faces = FacesT<D>;

// The global data of a face (its interface's alpha and functions), loaded
// by the first 4 M threads at the start of a kernel so that the loads are in
// flight with the mobility loads; prepare_faces completes the face data once
// the cell mobilities are in LDS.
template <int DD>
struct FaceLoadT {
  int e = -1;
  double al = 0.0;
  double phi[DD] = {};
};

template <int DD = D>
__device__ inline FaceLoadT<DD> load_faces(const SubArgs& a, int I, int J) {
  FaceLoadT<DD> fl;
  const int l = threadIdx.x;
  if (l < 4 * M) {
    const int side = l >> 4, t = l & 15;
    fl.e = side_iface(a.g, I, J, side);
    // loaded from selected addresses (the first permeability stands in on
    // the domain boundary), so that the loads are not behind a branch
    const bool has = fl.e >= 0;
    const double al = *(has ? a.alpha + fl.e : a.K);
    double ph[DD];
#pragma unroll
    for (int k = 0; k < DD; ++k) ph[k] = *(has ? a.basis + ((size_t)fl.e * DD + k) * M + t : a.K);
    fl.al = has ? al : 0.0;
#pragma unroll
    for (int k = 0; k < DD; ++k) fl.phi[k] = has ? ph[k] : 0.0;
  }
  return fl;
}

template <int DD>
__device__ inline void prepare_faces(const SubArgs& a, const FaceLoadT<DD>& fl, const double* kap,
                                     FacesT<DD>& f, int I, int J) {
  const Geo& g = a.g;
  const int l = threadIdx.x;
  if (l < 4 * M) {
    const int side = l >> 4, t = l & 15;
    double tr = 0.0, bt = 0.0, bl = 0.0, gr = 0.0;
    if (fl.e >= 0) {
      const SideGeo sg = side_geo(g, side);
      const int lc = side_cell<M>(side, t);
      const double kk = kap[lc];
      tr = sg.flen * kk / (sg.dist + fl.al * sg.H);
      bt = fl.al * sg.H / kk;
      bl = bt / sg.flen;
      if (a.rho) {
        gr = robin_grav(a, side, (size_t)(J * M + lc / M) * g.nx + I * M + lc % M, tr, sg.dist);
      }
    }
    f.gr[side][t] = gr;
    f.tr[side][t] = tr;
    f.bt[side][t] = bt;
    f.bl[side][t] = bl;
#pragma unroll
    for (int k = 0; k < DD; ++k) f.phi[side][k][t] = fl.phi[k];
  }
}

// Robin data of the basis columns of one window of 4 dofs per side (dofs
// 4 win .. 4 win + 3), bside[side][t][k] = T_R g_{4 win + k}(t) (flux
// functions scaled by -beta sigma), from the face data (first 4 M threads).
template <int DD>
__device__ inline void robin_data(const Geo& g, const FacesT<DD>& f, double (*bside)[M][4], int win = 0) {
  const int l = threadIdx.x;
  if (l < 4 * M) {
    const int side = l >> 4, t = l & 15;
    const double sig = side_sigma(side);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int kg = 4 * win + k;
      const double ph = f.phi[side][kg][t];
      bside[side][t][k] = f.tr[side][t] * (kg < g.nP ? ph : -f.bt[side][t] * sig * ph);
    }
  }
}

// Traces of the columns of one window on the skeleton faces (xb: solution in
// the cells next to each side's faces; column 0 the particular solution,
// column 1 + c the window's basis column c, which is dof 4 win + (c & 3) of
// side c >> 2) projected on all DD interface functions of each side: the
// window's columns of the subdomain's block of the interface system, rows
// of flux dofs negated (the form in which the assembled interface matrix is
// symmetric), last column = right-hand side (written by window 0).  One
// (side, column) pair per thread, the DD rows of that side accumulated
// together.  Slots beyond an interface's functions (nact) get a zero row and
// column, and 1 on the diagonal from the lower-index side (the dof is then
// 0), as in the per-subdomain kernels.
template <int DD>
__device__ inline void write_block(const SubArgs& a, int sd, int I, int J, const FacesT<DD>& f,
                                   const double (*xb)[M][R], int win = 0) {
  const Geo& g = a.g;
  constexpr int NBR = 4 * DD, NBC = 4 * DD + 1;
  constexpr int NQ = 17;                       // window columns + right-hand side
  double* blk = a.blocks + (size_t)sd * NBR * NBC;
  const int nP = g.nP;
  int e0side = -1;
  bool e0lo = false;
  if (g.gauge) {
    for (int side = 0; side < 4; ++side)
      if (side_iface(g, I, J, side) == 0) { e0side = side; e0lo = side_sigma(side) > 0; }
  }
  const int npair = win == 0 ? 4 * NQ : 4 * (NQ - 1);
  for (int pr = threadIdx.x; pr < npair; pr += blockDim.x) {
    const int side = pr / (npair / 4), ql = pr % (npair / 4);
    const bool rhs = ql == NQ - 1;
    const int col = rhs ? 0 : 1 + ql;                             // column of xb
    const int csd = ql >> 2, kc = 4 * win + (ql & 3);             // the column's side and dof
    const int qc = rhs ? NBR : csd * DD + kc;                     // its column of the block
    const int e = side_iface(g, I, J, side);
    double acc[DD];
#pragma unroll
    for (int k = 0; k < DD; ++k) acc[k] = 0.0;
    const double sig = side_sigma(side);
    if (e >= 0) {
      const bool colside = !rhs && csd == side;
      const bool flux_col = colside && kc >= nP;
      const double gscale = colside ? 1.0 : 0.0;
      const int kp = colside ? kc : 0;
#pragma unroll 4
      for (int t = 0; t < M; ++t) {
        const double ph = f.phi[side][kp][t];
        const double gv = gscale * (flux_col ? -f.bt[side][t] * sig * ph : ph);
        const double F = f.tr[side][t] * (xb[side][t][col] - gv) + (rhs ? f.gr[side][t] : 0.0);
        const double wu = fma(f.bl[side][t], F, gv);
#pragma unroll
        for (int k = 0; k < DD; ++k) acc[k] = fma(f.phi[side][k][t], k < nP ? F : wu, acc[k]);
      }
    }
    const double flen = side_geo(g, side).flen;
    const int es = rhs ? -1 : side_iface(g, I, J, csd);
    const bool col_dead = a.nact && es >= 0 && !slot_active(a, es, kc);
#pragma unroll
    for (int k = 0; k < DD; ++k) {
      const int r = side * DD + k;
      double val = 0.0;
      if (e >= 0) {
        const double natural = (k < nP) ? acc[k] : sig * flen * acc[k];
        const double sgn = (k < nP) ? 1.0 : -1.0;
        val = !rhs ? sgn * natural : -sgn * natural;
        if (e0side >= 0) {
          const int r0 = e0side * DD;
          if (r == r0) val = (qc == r0 && e0lo) ? 1.0 : 0.0;
          else if (qc == r0) val = 0.0;
        }
        if (a.nact) {
          if (!slot_active(a, e, k)) val = (qc == r && sig > 0) ? 1.0 : 0.0;
          else if (col_dead) val = 0.0;
        }
      }
      blk[r * NBC + qc] = val;
    }
  }
}

// ---------------------------------------------------------------------------
// Basis functions by two wavefronts per subdomain: wave 0 eliminates block
// rows 0..MID-1 downwards and solves the joining row MID, wave 1 eliminates
// rows M-1..MID+1 upwards.  Each wavefront keeps only its own rows' inverse
// blocks and solution tiles in registers, so two wavefronts fit on a SIMD,
// and the two chains run on different SIMDs.  The waves exchange the tiles
// next to the joining row through LDS; everything else of a row is local to
// the wave that owns it (LDS written and read by the same wavefront needs no
// barrier: its LDS accesses complete in program order).
// ---------------------------------------------------------------------------
constexpr int PAIR = 2 * WAVE;
static_assert(MM % PAIR == 0, "whole cells per thread");
constexpr int NU = MID + 1;       // rows of wave 0: 0 .. MID
constexpr int NL = M - 1 - MID;   // rows of wave 1: M-1 .. MID+1 (index t is row M-1-t)

// DD dofs per interface side: DD / 4 windows of 4 dofs per side, one
// work-group each (work-group b: subdomain b / (DD / 4), window b % (DD / 4)).
// Every window factorises the subdomain's matrix, solves its 16 basis columns
// and the particular solution (stored by window 0), and writes its columns
// of the interface block.
template <bool LIST, int DD>
__global__ void __launch_bounds__(PAIR, 2) basis_pair_kernel(SubArgs a) {
  static_assert(DD % 4 == 0 && (!LIST || DD == 4), "windows of 4 dofs per side");
  constexpr int NW = DD / 4, RX = 4 * DD + 1;
  __shared__ double kap[MM], dg[MM], ex[MM], cy[MM], b0[MM], pz[MM];
  __shared__ float dgl[MM];            // rounding error of the diagonal sums
  __shared__ FacesT<DD> fc;
  __shared__ double bside[4][M][D];
  __shared__ double xb[4][M][R];
  __shared__ double xs[2][M][M + 1];   // exchange tiles; per-wave staging
  __shared__ double zc[MM], rpz[MM];
  const Geo& g = a.g;
  // the wave index is uniform per wavefront: taken into a scalar register,
  // so that row offsets that depend on it are scalar too
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63, c = lane & 15, gq = lane >> 4;
  int sd = NW == 1 ? (int)blockIdx.x : (int)blockIdx.x / NW;
  const int win = NW == 1 ? 0 : (int)blockIdx.x % NW;
  if (LIST) {   // re-solve only the subdomains on the fallback list
    if ((int)blockIdx.x >= a.fallback[0]) return;
    sd = a.fallback[1 + blockIdx.x];
  }
  const int I = sd % g.SX, J = sd / g.SX;

  const FaceLoadT<DD> fl = load_faces<DD>(a, I, J);
  CellLoads cl[MM / PAIR];   // issued with the permeability loads
#pragma unroll
  for (int q = 0; q < MM / PAIR; ++q) cl[q] = cell_loads<M>(a, I, J, tid + PAIR * q, 1);
  load_kappa<M>(a, I, J, kap);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MM / PAIR; ++q)
    assemble_cell<M, 1, false>(a, I, J, tid + PAIR * q, kap, dg, ex, cy, b0 + tid + PAIR * q, 1, nullptr,
                               cl[q], dgl);
  prepare_faces(a, fl, kap, fc, I, J);
  __syncthreads();
  robin_data(g, fc, bside, win);
  __syncthreads();

  const d4 zero = {0.0, 0.0, 0.0, 0.0};
  const int nchain = w ? NL : MID;   // rows eliminated before the join
  d4 Sv[NU], Xv[NU];
  PivotCheck pvc;
  d4 pc = zero;   // particular column carried along the chain
#pragma unroll
  for (int t = 0; t < MID; ++t) {
    if (t < nchain) {
      const int j = w ? M - 1 - t : t;
      const int jc = w ? j : j - 1;     // coupling towards the chain's previous row
      d4 s = coupled_block(j, t > 0 ? jc : -1, t > 0 ? Sv[t > 0 ? t - 1 : 0] : zero, c, gq, dg, ex, cy);
      s = gauss_jordan16(s, c, gq, pvc);
      Sv[t] = s;
      d4 r, rp;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 4 * v + gq;
        double bv = side_rhs(bside, j, row, c), bp = b0[j * M + row];
        if (t > 0) {
          const double cc = cy[jc * M + row];
          bv -= cc * Xv[t > 0 ? t - 1 : 0][v];
          bp -= cc * pc[v];
        }
        r[v] = bv;
        rp[v] = bp;
      }
      d4 z = zero, zz = zero;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        z = mfma(s[kk], r[kk], z);
        zz = mfma(s[kk], rp[kk], zz);
      }
      Xv[t] = z;
      pc = zz;
      if (c == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) pz[j * M + 4 * v + gq] = zz[v];
      }
    }
  }
  // join: wave 1 hands over its last inverse block and forward tile (row
  // MID+1); wave 0 solves row MID and hands back its solution tile
  if (w == 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      xs[0][4 * v + gq][c] = Sv[NL - 1][v];
      xs[1][4 * v + gq][c] = Xv[NL - 1][v];
    }
  }
  __syncthreads();
  if (w == 0) {
    constexpr int j = MID;
    d4 s = coupled_block(j, j - 1, Sv[MID - 1], c, gq, dg, ex, cy);
    d4 r, rp;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * v + gq;
      s[v] -= cy[j * M + row] * xs[0][row][c] * cy[j * M + c];
      const double cu = cy[(j - 1) * M + row], cl = cy[j * M + row];
      r[v] = side_rhs(bside, j, row, c) - cu * Xv[MID - 1][v] - cl * xs[1][row][c];
      rp[v] = b0[j * M + row] - cu * pc[v] - cl * pz[(j + 1) * M + row];
    }
    s = gauss_jordan16(s, c, gq, pvc);
    Sv[MID] = s;
    d4 z = zero, zz = zero;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      z = mfma(s[kk], r[kk], z);
      zz = mfma(s[kk], rp[kk], zz);
    }
    Xv[MID] = z;
    if (c == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) pz[j * M + 4 * v + gq] = zz[v];
    }
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) xs[0][4 * v + gq][c] = Xv[MID][v];
  }
  __syncthreads();
  d4 xm;      // solution tile of the joining row, in both waves
#pragma unroll
  for (int v = 0; v < 4; ++v) xm[v] = (w == 0) ? Xv[MID][v] : xs[0][4 * v + gq][c];
  // back substitution outwards from the joining row
  {
    d4 xp = xm;
#pragma unroll
    for (int v = 0; v < 4; ++v) pc[v] = pz[MID * M + 4 * v + gq];
#pragma unroll
    for (int t = MID - 1; t >= 0; --t) {
      if (t < nchain) {
        const int j = w ? M - 1 - t : t;
        const int jc = w ? j - 1 : j;   // coupling towards the joining side
        d4 tt, tp, xq;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = 4 * v + gq;
          const double cc = -cy[jc * M + row];
          tt[v] = cc * xp[v];
          tp[v] = cc * pc[v];
          xq[v] = pz[j * M + row];
        }
        d4 x = Xv[t];
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          x = mfma(Sv[t][kk], tt[kk], x);
          xq = mfma(Sv[t][kk], tp[kk], xq);
        }
        Xv[t] = x;
        xp = x;
        pc = xq;
        if (c == 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) pz[j * M + 4 * v + gq] = xq[v];
        }
      }
    }
  }
  if (pvc.bad()) atomicOr(a.status, ST_LOCAL_PIVOT);

  // one step of iterative refinement of all 17 columns (residual in
  // double-double, correction by the same two-chain sweeps).  With a plain
  // FP64 residual the parity with the oracle is the same, but the interface
  // blocks then keep an asymmetry near 1e-13 of their size, which the
  // interface elimination (symmetric diagonal-block inverses) turns into a
  // residual above its refinement threshold on some steps
  __syncthreads();
  for (int l = tid; l < MM; l += PAIR) {
    const int i = l % M, j = l / M;
    double ph = b0[l], pl = 0.0;
    dd_fma(ph, pl, -dg[l], pz[l]);
    dd_fma_low(pl, -(double)dgl[l], pz[l]);
    dd_fma(ph, pl, i < M - 1 ? -ex[l] : 0.0, pz[i < M - 1 ? l + 1 : l]);
    dd_fma(ph, pl, i > 0 ? -ex[l - 1] : 0.0, pz[i > 0 ? l - 1 : l]);
    dd_fma(ph, pl, j < M - 1 ? -cy[l] : 0.0, pz[j < M - 1 ? l + M : l]);
    dd_fma(ph, pl, j > 0 ? -cy[l - M] : 0.0, pz[j > 0 ? l - M : l]);
    rpz[l] = ph + pl;
  }
  if (w == 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) xs[1][4 * v + gq][c] = Xv[NL - 1][v];
  }
  __syncthreads();
  d4 xo;      // the other wave's tile next to the join (rows MID+1 / MID)
#pragma unroll
  for (int v = 0; v < 4; ++v) xo[v] = (w == 0) ? xs[1][4 * v + gq][c] : xm[v];
  __syncthreads();
  double (*T)[M + 1] = xs[w];   // per-wave staging of in-row neighbours
  // residual of own row index t (row j): neighbours along y from the
  // chain's tiles, the other wave's tile across the join
  auto residual = [&](int t, int j, d4& r) {
#pragma unroll
    for (int v = 0; v < 4; ++v) T[4 * v + gq][c] = Xv[t][v];
    __builtin_amdgcn_wave_barrier();
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * v + gq, l = j * M + i;
      double hi = side_rhs(bside, j, i, c), lo = 0.0;
      dd_fma(hi, lo, -dg[l], Xv[t][v]);
      dd_fma_low(lo, -(double)dgl[l], Xv[t][v]);
      dd_fma(hi, lo, i < M - 1 ? -ex[l] : 0.0, T[i < M - 1 ? i + 1 : i][c]);
      dd_fma(hi, lo, i > 0 ? -ex[i > 0 ? l - 1 : l] : 0.0, T[i > 0 ? i - 1 : i][c]);
      r[v] = hi + lo;
    }
    __builtin_amdgcn_wave_barrier();
  };
  f4z Zc[NU];
  d4 qc = zero;   // particular correction carried along the chain
#pragma unroll
  for (int t = 0; t < MID; ++t) {
    if (t < nchain) {
      const int j = w ? M - 1 - t : t;
      const int jc = w ? j : j - 1;
      d4 r;
      residual(t, j, r);
      // y neighbours: the previous row of the chain (t-1) and the next (t+1,
      // or across the join for the last row before it)
      const int jcn = w ? j - 1 : j;                // coupling towards the join
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * v + gq;
        double hi = r[v], lo = 0.0;
        const double xnext = (t + 1 < nchain) ? Xv[t + 1 < NU ? t + 1 : t][v] : (w ? xm[v] : Xv[MID][v]);
        dd_fma(hi, lo, -cy[jcn * M + i], xnext);
        if (t > 0) dd_fma(hi, lo, -cy[jc * M + i], Xv[t > 0 ? t - 1 : 0][v]);
        r[v] = hi + lo;
      }
      d4 rp;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int i = 4 * v + gq;
        rp[v] = rpz[j * M + i];
        if (t > 0) {
          const double cc = cy[jc * M + i];
          r[v] -= cc * (double)Zc[t > 0 ? t - 1 : 0][v];
          rp[v] -= cc * qc[v];
        }
      }
      d4 z = zero, zz = zero;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) {
        z = mfma(Sv[t][kk], r[kk], z);
        zz = mfma(Sv[t][kk], rp[kk], zz);
      }
      Zc[t] = tof(z);
      qc = zz;
      if (c == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) zc[j * M + 4 * v + gq] = zz[v];
      }
    }
  }
  // join of the correction sweeps
  if (w == 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) xs[1][4 * v + gq][c] = (double)Zc[NL - 1][v];
  }
  __syncthreads();
  if (w == 0) {
    constexpr int j = MID;
    d4 r;
    residual(MID, j, r);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * v + gq;
      double hi = r[v], lo = 0.0;
      dd_fma(hi, lo, -cy[j * M + i], xo[v]);
      dd_fma(hi, lo, -cy[(j - 1) * M + i], Xv[MID - 1][v]);
      r[v] = hi + lo;
    }
    d4 rp;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int i = 4 * v + gq;
      const double cu = cy[(j - 1) * M + i], cl = cy[j * M + i];
      r[v] -= cu * (double)Zc[MID - 1][v] + cl * xs[1][i][c];
      rp[v] = rpz[j * M + i] - cu * qc[v] - cl * zc[(j + 1) * M + i];
    }
    d4 z = zero, zz = zero;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      z = mfma(Sv[MID][kk], r[kk], z);
      zz = mfma(Sv[MID][kk], rp[kk], zz);
    }
    Zc[MID] = tof(z);
    if (c == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) zc[j * M + 4 * v + gq] = zz[v];
    }
  }
  __syncthreads();
  if (w == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) xs[0][4 * v + gq][c] = (double)Zc[MID][v];
  }
  __syncthreads();
  {
    d4 cm;
#pragma unroll
    for (int v = 0; v < 4; ++v) cm[v] = xs[0][4 * v + gq][c];
    if (w == 0) Xv[MID] += cm;
    if (w == 0 && c == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) pz[MID * M + 4 * v + gq] += zc[MID * M + 4 * v + gq];
    }
    d4 cp = cm, qp;
#pragma unroll
    for (int v = 0; v < 4; ++v) qp[v] = zc[MID * M + 4 * v + gq];
#pragma unroll
    for (int t = MID - 1; t >= 0; --t) {
      if (t < nchain) {
        const int j = w ? M - 1 - t : t;
        const int jc = w ? j - 1 : j;
        d4 tt, tq, xq;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int i = 4 * v + gq;
          const double cc = -cy[jc * M + i];
          tt[v] = cc * cp[v];
          tq[v] = cc * qp[v];
          xq[v] = zc[j * M + i];
        }
        d4 x = tod(Zc[t]);
#pragma unroll
        for (int kk = 0; kk < 4; ++kk) {
          x = mfma(Sv[t][kk], tt[kk], x);
          xq = mfma(Sv[t][kk], tq[kk], xq);
        }
        cp = x;
        qp = xq;
        Xv[t] += x;
        if (c == 0) {
#pragma unroll
          for (int v = 0; v < 4; ++v) pz[j * M + 4 * v + gq] += xq[v];
        }
      }
    }
  }
  __syncthreads();

  // basis functions to global memory, column-major per subdomain: each
  // row tile is transposed through the wave's LDS tile so that every store
  // instruction writes four whole 128-byte column segments (tile column
  // q0 + 4 s4 is dof 4 win + q0 of side s4)
  double* Xg = a.X + (size_t)sd * RX * MM;
  {
    double (*Tt)[M + 1] = xs[w];
    const int ci = lane & 15, q0 = lane >> 4;
#pragma unroll
    for (int t = 0; t < NU; ++t) {
      if (t < nchain || (w == 0 && t == MID)) {
        const int j = w ? M - 1 - t : t;
#pragma unroll
        for (int v = 0; v < 4; ++v) Tt[4 * v + gq][c] = Xv[t][v];
        __builtin_amdgcn_wave_barrier();
#pragma unroll
        for (int s4 = 0; s4 < 4; ++s4) {
          const int q = q0 + 4 * s4;
          const int qg = NW == 1 ? q : s4 * DD + 4 * win + q0;   // (the same index for NW = 1,
                                                                  // in the form that keeps spills down)
          // streaming stores: the stitch reads X back in another launch, and
          // lines kept in L2 would only push out the spilled registers
          __builtin_nontemporal_store(Tt[ci][q], &Xg[(size_t)(1 + qg) * MM + j * M + ci]);
        }
        __builtin_amdgcn_wave_barrier();
        if (gq == 0) xb[0][j][1 + c] = Xv[t][0];
        if (gq == 3) xb[1][j][1 + c] = Xv[t][3];
      }
    }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    if (w == 0) xb[2][4 * v + gq][1 + c] = Xv[0][v];
    else xb[3][4 * v + gq][1 + c] = Xv[0][v];
  }
  if (win == 0)
    for (int l = tid; l < MM; l += PAIR) __builtin_nontemporal_store(pz[l], &Xg[l]);
  if (tid < M) {
    xb[0][tid][0] = pz[tid * M];
    xb[1][tid][0] = pz[tid * M + M - 1];
    xb[2][tid][0] = pz[tid];
    xb[3][tid][0] = pz[(M - 1) * M + tid];
  }
  __syncthreads();
  write_block(a, sd, I, J, fc, xb, win);
}

// Two-wavefront elimination of the 16 Schur blocks (wave 0: rows 0..MID-1
// and the joining row MID, wave 1: rows M-1..MID+1, index t = row M-1-t);
// xch is an LDS tile for the hand-over at the join.  Both waves must call.
// TAG (the caller's dofs per side) gives each stitch kernel a copy of its
// own: a helper with one caller compiles to fewer spills in that caller.
template <int TAG>
__device__ inline void factor_pair(d4* Sv, int w, int c, int g, const double* dg, const double* ex,
                                   const double* cy, double (*xch)[M + 1], PivotCheck& pvc) {
  const d4 zero = {0.0, 0.0, 0.0, 0.0};
  const int nchain = w ? NL : MID;
#pragma unroll
  for (int t = 0; t < MID; ++t) {
    if (t < nchain) {
      const int j = w ? M - 1 - t : t;
      const int jc = w ? j : j - 1;
      d4 s = coupled_block(j, t > 0 ? jc : -1, t > 0 ? Sv[t > 0 ? t - 1 : 0] : zero, c, g, dg, ex, cy);
      Sv[t] = gauss_jordan16(s, c, g, pvc);
    }
  }
  if (w == 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) xch[4 * v + g][c] = Sv[NL - 1][v];
  }
  __syncthreads();
  if (w == 0) {
    constexpr int j = MID;
    d4 s = coupled_block(j, j - 1, Sv[MID - 1], c, g, dg, ex, cy);
#pragma unroll
    for (int v = 0; v < 4; ++v) s[v] -= cy[j * M + 4 * v + g] * xch[4 * v + g][c] * cy[j * M + c];
    Sv[MID] = gauss_jordan16(s, c, g, pvc);
  }
  __syncthreads();
}

// One column solve with the blocks of factor_pair (rhs and result in LDS,
// cell-major; the column is replicated over the 16 MFMA columns and lanes
// with c == 0 write the result).  Both waves must call.
template <int TAG>
__device__ inline void solve_column_pair(const d4* Sv, int w, const double* rhs, double* out, int c,
                                         int g, const double* cy) {
  const d4 zero = {0.0, 0.0, 0.0, 0.0};
  const int nchain = w ? NL : MID;
  d4 zc = zero;
#pragma unroll
  for (int t = 0; t < MID; ++t) {
    if (t < nchain) {
      const int j = w ? M - 1 - t : t;
      const int jc = w ? j : j - 1;
      d4 r;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 4 * v + g;
        double b = rhs[j * M + row];
        if (t > 0) b -= cy[jc * M + row] * zc[v];
        r[v] = b;
      }
      d4 acc = zero;
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) acc = mfma(Sv[t][kk], r[kk], acc);
      zc = acc;
      if (c == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) out[j * M + 4 * v + g] = acc[v];
      }
    }
  }
  __syncthreads();
  if (w == 0) {
    constexpr int j = MID;
    d4 r;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * v + g;
      r[v] = rhs[j * M + row] - cy[(j - 1) * M + row] * zc[v] - cy[j * M + row] * out[(j + 1) * M + row];
    }
    d4 acc = zero;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) acc = mfma(Sv[MID][kk], r[kk], acc);
    if (c == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) out[j * M + 4 * v + g] = acc[v];
    }
  }
  __syncthreads();
  d4 xp;
#pragma unroll
  for (int v = 0; v < 4; ++v) xp[v] = out[MID * M + 4 * v + g];
#pragma unroll
  for (int t = MID - 1; t >= 0; --t) {
    if (t < nchain) {
      const int j = w ? M - 1 - t : t;
      const int jc = w ? j - 1 : j;
      d4 tt, x;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = 4 * v + g;
        tt[v] = -cy[jc * M + row] * xp[v];
        x[v] = out[j * M + row];
      }
#pragma unroll
      for (int kk = 0; kk < 4; ++kk) x = mfma(Sv[t][kk], tt[kk], x);
      xp = x;
      if (c == 0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) out[j * M + 4 * v + g] = x[v];
      }
    }
  }
  __syncthreads();
}

// ---------------------------------------------------------------------------
// FP32 factors and solves with FP64 iterative refinement (16 x 16, 2 + 2 dofs)
// ---------------------------------------------------------------------------
//
// The local matrix is scaled symmetrically, A^ = Ds A Ds with Ds = diag(A)^-1/2,
// which removes the permeability scale from the FP32 factorisation.  The
// Schur blocks of A^ are inverted in FP32 (Gauss-Jordan in registers), and
// both block sweeps run on v_mfma_f32_16x16x4f32, whose output layout puts
// rows 4g .. 4g+3 of column c in lane c + 16 g (measured on the device).  The
// solution is kept in FP64; every refinement step forms R = B - A X in
// double-double with the exact diagonal (the cells' mass balances; an FP64
// residual or a rounded diagonal would leave local solutions conservative
// only to eps T |x| per cell, which the stitch inherits), solves
// A^ y = Ds R in FP32 and adds Ds y.  A subdomain whose correction does
// not fall below IR_DONE of its solution within IR_MAX steps, or whose FP32
// pivots fail, is appended to a.fallback and re-solved in FP64 (IR_DONE and
// IR_MAX are a.ir_tol and a.ir_max, by default 1e-12 and 8 steps).  The
// error left after a step is about the contraction factor times that step's
// correction, so IR_DONE = 1e-12 leaves local errors near FP64 accuracy.

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ inline float readlane_f(float x, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), lane));
}

__device__ inline f4 mfma32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <int K>
__device__ inline float row_bcast_f(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), 0x150 + K, 0xF, 0xF, false));
}

// One FP32 Gauss-Jordan sweep with pivot K (f32 output layout: lane c + 16 g
// holds rows 4 g .. 4 g + 3 of column c): the pivot column comes from lane K
// of the lane's own 16-lane row, the pivot row from lane c + 16 (K / 4).
// 1/p is the hardware reciprocal (1 ulp in FP32; the refinement in FP64
// absorbs it).  pmin accumulates the smallest pivot (NaN-free pivots that are
// all positive leave it positive; a NaN pivot makes it NaN through pnan).
template <int K>
__device__ inline void gj_sweep_f32(f4& s, int c, int g, float& pmin, float& pnan) {
  constexpr int kg = K >> 2, kv = K & 3;
  const float p = readlane_f(s[kv], K + 16 * kg);
  const float prow = __shfl(s[kv], c + 16 * kg);
  float pcol[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) pcol[v] = row_bcast_f<K>(s[v]);
  {
    float r;   // the plain v_min_f32 (a NaN pivot is caught by pnan)
    asm("v_min_f32 %0, %1, %2" : "=v"(r) : "v"(pmin), "s"(p));
    pmin = r;
  }
  pnan = fmaf(p, 0.0f, pnan);
  const float ip = __builtin_amdgcn_rcpf(p);
  const float b = (c == K) ? ip : prow * ip;
  const float keep = (c == K) ? 0.0f : 1.0f;   // column K is replaced, not updated
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float nv = fmaf(-pcol[v], b, s[v] * keep);
    s[v] = (v == kv && g == kg) ? b : nv;
  }
}

template <int K>
struct GJ16F {
  static __device__ inline void run(f4& s, int c, int g, float& pmin, float& pnan) {
    gj_sweep_f32<K>(s, c, g, pmin, pnan);
    GJ16F<K + 1>::run(s, c, g, pmin, pnan);
  }
};
template <>
struct GJ16F<M> {
  static __device__ inline void run(f4&, int, int, float&, float&) {}
};

__device__ inline f4 gauss_jordan16_f32(f4 s, int c, int g, float& pmin, float& pnan) {
  GJ16F<0>::run(s, c, g, pmin, pnan);
  asm volatile("" : "+v"(pmin), "+v"(pnan));
  return s;
}

// scaled coupling between block rows j and j+1 at cell row i
__device__ inline double chat(const double* cy, const double* dsc, int j, int i) {
  return cy[j * M + i] * dsc[j * M + i] * dsc[(j + 1) * M + i];
}

// scaled diagonal block of row j (unit diagonal) minus C P C with C the
// scaled coupling of row jc (jc < 0: none), f32 output layout
__device__ inline f4 coupled_block32(int j, int jc, const f4& P, int c, int gq, const double* ex,
                                     const double* cy, const double* dsc) {
  f4 s;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const int row = 4 * gq + v, l = j * M + row;
    const double d = (row == c) ? 1.0
                   : (row == c + 1) ? ex[j * M + c] * dsc[j * M + c] * dsc[l]
                   : (c == row + 1) ? ex[l] * dsc[l] * dsc[j * M + c] : 0.0;
    float sv = (float)d;
    if (jc >= 0) sv -= (float)chat(cy, dsc, jc, row) * P[v] * (float)chat(cy, dsc, jc, c);
    s[v] = sv;
  }
  return s;
}

__device__ inline double wave_max(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  return v;
}

// Rows of the two elimination chains: wave W = 0 owns block rows 0..MID
// (index t = row) and solves the joining row MID, wave W = 1 owns rows
// M-1..MID+1 (index t = M-1-row).  Instantiating the per-wave code for each
// W makes every row index a compile-time constant (LDS offsets fold into the
// instructions, no per-row branches).
template <int W>
struct Chain {
  static constexpr int NR = W ? NL : NU;   // rows the wave owns
  static constexpr int NC = W ? NL : MID;  // rows it eliminates before the join
  static constexpr int row(int t) { return W ? M - 1 - t : t; }
  // coupling (row of cy) towards the previous row of the chain / the join
  static constexpr int cprev(int t) { return W ? M - 1 - t : t - 1; }
  static constexpr int cnext(int t) { return W ? M - 2 - t : t; }
};

// LDS of the FP32 + refinement kernel
struct Lds32 {
  double kap[MM], dg[MM], ex[MM], cy[MM], b0[MM], dsc[MM], px[MM];
  float dgl[MM];            // rounding error of the diagonal sums
  double bside[4][M][D];
  double xb[4][M][R];
  Faces fc;
  double T[2][M][M + 1];    // per-wave staging of in-row neighbours
  double xj[2][M][M + 1];   // solution tiles next to the join
  float xf[M][M + 1];       // FP32 hand-over tile at the join
  float pcol[MM];           // particular column (FP32 right-hand side / solution)
  double red[2][2];
  int bad[2];               // per wave: a pivot of its chain was not positive
};

// FP32 inverse Schur blocks of the scaled matrix along the wave's chain; the
// joining row is inverted by wave 0.  Both waves call.
template <int W>
__device__ inline void factor32(f4* Sv, Lds32& sh, int c, int gq, float& pmin, float& pnan) {
  using C = Chain<W>;
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int t = 0; t < C::NC; ++t) {
    const f4 s = coupled_block32(C::row(t), t > 0 ? C::cprev(t) : -1, t > 0 ? Sv[t > 0 ? t - 1 : 0] : zero,
                                 c, gq, sh.ex, sh.cy, sh.dsc);
    Sv[t] = gauss_jordan16_f32(s, c, gq, pmin, pnan);
  }
  if (W == 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) sh.xf[4 * gq + v][c] = Sv[NL - 1][v];
  }
  __syncthreads();
  if (W == 0) {
    constexpr int j = MID;
    f4 s = coupled_block32(j, j - 1, Sv[MID - 1], c, gq, sh.ex, sh.cy, sh.dsc);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * gq + v;
      s[v] -= (float)chat(sh.cy, sh.dsc, j, row) * sh.xf[row][c] * (float)chat(sh.cy, sh.dsc, j, c);
    }
    Sv[MID] = gauss_jordan16_f32(s, c, gq, pmin, pnan);
  }
  __syncthreads();
}

// Two-chain FP32 solve of the scaled system.  rhs(t) gives the 16 basis
// right-hand-side tile of the wave's row t; it is called in chain order, just
// before the row is eliminated (so a residual can be formed row by row).
// Wt[t] receives the solution.  sh.pcol: the particular right-hand side on
// entry, its solution on return (a second MFMA tile with the column
// replicated over its 16 columns; lanes with c == 0 write it).  Both waves
// call.
template <int W, class Rhs>
__device__ inline void solve32(const f4* Sv, f4* Wt, Lds32& sh, int c, int gq, Rhs rhs) {
  using C = Chain<W>;
  const double* cy = sh.cy;
  const double* dsc = sh.dsc;
  float* pcol = sh.pcol;
  const f4 zero = {0.f, 0.f, 0.f, 0.f};
  f4 pc = zero;
#pragma unroll
  for (int t = 0; t < C::NC; ++t) {
    const int j = C::row(t);
    f4 r = rhs(t), rp;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * gq + v;
      rp[v] = pcol[j * M + row];
      if (t > 0) {
        const float cc = (float)chat(cy, dsc, C::cprev(t), row);
        r[v] -= cc * Wt[t > 0 ? t - 1 : 0][v];
        rp[v] -= cc * pc[v];
      }
    }
    f4 z = zero, zz = zero;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      z = mfma32(Sv[t][kk], r[kk], z);
      zz = mfma32(Sv[t][kk], rp[kk], zz);
    }
    Wt[t] = z;
    pc = zz;
    if (c == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) pcol[j * M + 4 * gq + v] = zz[v];
    }
  }
  if (W == 1) {
#pragma unroll
    for (int v = 0; v < 4; ++v) sh.xf[4 * gq + v][c] = Wt[NL - 1][v];
  }
  __syncthreads();
  if (W == 0) {
    constexpr int j = MID;
    f4 r = rhs(MID), rp;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * gq + v;
      const float cu = (float)chat(cy, dsc, j - 1, row), cl = (float)chat(cy, dsc, j, row);
      r[v] -= cu * Wt[MID - 1][v] + cl * sh.xf[row][c];
      rp[v] = pcol[j * M + row] - cu * pc[v] - cl * pcol[(j + 1) * M + row];
    }
    f4 z = zero, zz = zero;
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      z = mfma32(Sv[MID][kk], r[kk], z);
      zz = mfma32(Sv[MID][kk], rp[kk], zz);
    }
    Wt[MID] = z;
    if (c == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) pcol[j * M + 4 * gq + v] = zz[v];
    }
  }
  __syncthreads();
  if (W == 0) {
#pragma unroll
    for (int v = 0; v < 4; ++v) sh.xf[4 * gq + v][c] = Wt[MID][v];
  }
  __syncthreads();
  f4 xp;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    xp[v] = W == 0 ? Wt[MID][v] : sh.xf[4 * gq + v][c];
    pc[v] = pcol[MID * M + 4 * gq + v];
  }
#pragma unroll
  for (int t = C::NC - 1; t >= 0; --t) {
    const int j = C::row(t);
    f4 tt, tp, xq;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * gq + v;
      const float cc = -(float)chat(cy, dsc, C::cnext(t), row);
      tt[v] = cc * xp[v];
      tp[v] = cc * pc[v];
      xq[v] = pcol[j * M + row];
    }
    f4 x = Wt[t];
#pragma unroll
    for (int kk = 0; kk < 4; ++kk) {
      x = mfma32(Sv[t][kk], tt[kk], x);
      xq = mfma32(Sv[t][kk], tp[kk], xq);
    }
    Wt[t] = x;
    xp = x;
    pc = xq;
    if (c == 0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) pcol[j * M + 4 * gq + v] = xq[v];
    }
  }
  __syncthreads();
}

// Double-double residual of the basis columns in the wave's row t, scaled and
// rounded to FP32 (the tile of the other wave next to the join must be in
// sh.xj).
template <int W>
__device__ inline f4 residual32_row(int t, const d4* Xv, Lds32& sh, int c, int gq) {
  using C = Chain<W>;
  const int j = C::row(t);
  double (*T)[M + 1] = sh.T[W];
#pragma unroll
  for (int v = 0; v < 4; ++v) T[4 * gq + v][c] = Xv[t][v];
  __builtin_amdgcn_wave_barrier();
  f4 w;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    // every load unconditional (indices clamped): the selects stay branch-free
    const int i = 4 * gq + v, l = j * M + i;
    const int ir = i < M - 1 ? i + 1 : i, il = i > 0 ? i - 1 : i;
    const double exr = sh.ex[l], exl = sh.ex[j * M + il];
    const double xr = T[ir][c], xl = T[il][c];
    // double-double, with the exact diagonal: the cells' mass balances
    double r = side_rhs(sh.bside, j, i, c), lo = 0.0;
    dd_fma(r, lo, -sh.dg[l], Xv[t][v]);
    dd_fma_low(lo, -(double)sh.dgl[l], Xv[t][v]);
    dd_fma(r, lo, i < M - 1 ? -exr : 0.0, xr);
    dd_fma(r, lo, i > 0 ? -exl : 0.0, xl);
    if (t > 0) dd_fma(r, lo, -sh.cy[C::cprev(t) * M + i], Xv[t > 0 ? t - 1 : 0][v]);
    const double xn = (t + 1 < C::NR) ? Xv[t + 1 < C::NR ? t + 1 : t][v] : sh.xj[1 - W][i][c];
    dd_fma(r, lo, -sh.cy[C::cnext(t) * M + i], xn);
    w[v] = (float)(sh.dsc[l] * (r + lo));
  }
  __builtin_amdgcn_wave_barrier();
  return w;
}

// FP32 factorisation + FP64 iterative refinement, two wavefronts per
// subdomain with the chains of basis_pair_kernel.  The local matrix is scaled
// symmetrically (Ds A Ds, Ds = diag(A)^-1/2, unit diagonal); the inverse
// Schur blocks and the correction solves are FP32 (MFMA with FP32
// accumulation), the solution FP64 and the residuals double-double.  Refinement stops when
// the largest correction is below a.ir_tol of the largest solution value; a
// subdomain that ends above it, or met a bad pivot, is listed for the
// FP64 re-solve.
template <int W>
__device__ inline void basis32_body(const SubArgs& a, Lds32& sh) {
  using C = Chain<W>;
  const Geo& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, c = lane & 15, gq = lane >> 4;
  const int sd = blockIdx.x;
  const int I = sd % g.SX, J = sd / g.SX;

  const FaceLoadT<D> fl = load_faces(a, I, J);
  CellLoads cl[MM / PAIR];   // issued with the permeability loads
#pragma unroll
  for (int q = 0; q < MM / PAIR; ++q) cl[q] = cell_loads<M>(a, I, J, tid + PAIR * q, 1);
  load_kappa<M>(a, I, J, sh.kap);
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MM / PAIR; ++q)
    assemble_cell<M, 1, false>(a, I, J, tid + PAIR * q, sh.kap, sh.dg, sh.ex, sh.cy,
                               sh.b0 + tid + PAIR * q, 1, nullptr, cl[q], sh.dgl);
  prepare_faces(a, fl, sh.kap, sh.fc, I, J);
  for (int l = tid; l < MM; l += PAIR) sh.dsc[l] = 1.0 / sqrt(sh.dg[l]);
  __syncthreads();
  robin_data(g, sh.fc, sh.bside);
  __syncthreads();

  f4 Sv[C::NR];
  float pmin = 1.0f, pnan = 0.0f;
  factor32<W>(Sv, sh, c, gq, pmin, pnan);
  if (lane == 0) sh.bad[W] = !(pmin > 0.0f) || pnan != 0.0f;

  // first solve: X = Ds A^-1 Ds B
  f4 Wt[C::NR];
  d4 Xv[C::NR];
  for (int l = tid; l < MM; l += PAIR) sh.pcol[l] = (float)(sh.dsc[l] * sh.b0[l]);
  __syncthreads();
  const bool bad = sh.bad[0] || sh.bad[1];
  solve32<W>(Sv, Wt, sh, c, gq, [&](int t) {
    const int j = C::row(t);
    f4 w;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int row = 4 * gq + v;
      w[v] = (float)(sh.dsc[j * M + row] * side_rhs(sh.bside, j, row, c));
    }
    return w;
  });
#pragma unroll
  for (int t = 0; t < C::NR; ++t) {
    const int j = C::row(t);
#pragma unroll
    for (int v = 0; v < 4; ++v) Xv[t][v] = sh.dsc[j * M + 4 * gq + v] * (double)Wt[t][v];
  }
  for (int l = tid; l < MM; l += PAIR) sh.px[l] = sh.dsc[l] * (double)sh.pcol[l];
  __syncthreads();

  // refinement: double-double residual (the cells' mass balances), FP32 correction
  int used = 0;
  double rel = 1.0;
#pragma unroll 1
  for (int it = 0; it < a.ir_max; ++it) {
#pragma unroll
    for (int v = 0; v < 4; ++v) sh.xj[W][4 * gq + v][c] = Xv[C::NR - 1][v];
    __syncthreads();
    for (int l = tid; l < MM; l += PAIR) {
      const int li = l % M, lj = l / M;
      const int le = li < M - 1 ? l + 1 : l, lw = li > 0 ? l - 1 : l;
      const int ln = lj < M - 1 ? l + M : l, ls = lj > 0 ? l - M : l;
      double r = sh.b0[l], lo = 0.0;
      dd_fma(r, lo, -sh.dg[l], sh.px[l]);
      dd_fma_low(lo, -(double)sh.dgl[l], sh.px[l]);
      dd_fma(r, lo, li < M - 1 ? -sh.ex[l] : 0.0, sh.px[le]);
      dd_fma(r, lo, li > 0 ? -sh.ex[lw] : 0.0, sh.px[lw]);
      dd_fma(r, lo, lj < M - 1 ? -sh.cy[l] : 0.0, sh.px[ln]);
      dd_fma(r, lo, lj > 0 ? -sh.cy[ls] : 0.0, sh.px[ls]);
      sh.pcol[l] = (float)(sh.dsc[l] * (r + lo));
    }
    __syncthreads();
    solve32<W>(Sv, Wt, sh, c, gq, [&](int t) { return residual32_row<W>(t, Xv, sh, c, gq); });
    double cmax = 0.0, xmax = 0.0;
#pragma unroll
    for (int t = 0; t < C::NR; ++t) {
      const int j = C::row(t);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double dx = sh.dsc[j * M + 4 * gq + v] * (double)Wt[t][v];
        Xv[t][v] += dx;
        cmax = fmax(cmax, fabs(dx));
        xmax = fmax(xmax, fabs(Xv[t][v]));
      }
    }
    for (int l = tid; l < MM; l += PAIR) {
      const double dx = sh.dsc[l] * (double)sh.pcol[l];
      sh.px[l] += dx;
      cmax = fmax(cmax, fabs(dx));
      xmax = fmax(xmax, fabs(sh.px[l]));
    }
    cmax = wave_max(cmax);
    xmax = wave_max(xmax);
    if (lane == 0) {
      sh.red[W][0] = cmax;
      sh.red[W][1] = xmax;
    }
    __syncthreads();
    cmax = fmax(sh.red[0][0], sh.red[1][0]);
    xmax = fmax(sh.red[0][1], sh.red[1][1]);
    __syncthreads();
    used = it + 1;
    rel = cmax / fmax(xmax, 1e-300);
    if (rel <= a.ir_tol) break;
  }
  if (W == 0 && tid == 0) {
    atomicMax(a.ir_iters, used);
    if (bad || !(rel <= a.ir_tol)) {
      const int q = atomicAdd(a.fallback, 1);
      a.fallback[1 + q] = sd;
    }
  }

  // basis functions to global memory (f32 layout: rows 4gq .. 4gq+3 of column c)
  double* Xg = a.X + (size_t)sd * R * MM;
#pragma unroll
  for (int t = 0; t < C::NR; ++t) {
    const int j = C::row(t);
#pragma unroll
    for (int v = 0; v < 4; ++v) Xg[(size_t)(1 + c) * MM + j * M + 4 * gq + v] = Xv[t][v];
    if (gq == 0) sh.xb[0][j][1 + c] = Xv[t][0];
    if (gq == 3) sh.xb[1][j][1 + c] = Xv[t][3];
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) sh.xb[W ? 3 : 2][4 * gq + v][1 + c] = Xv[0][v];
  for (int l = tid; l < MM; l += PAIR) Xg[l] = sh.px[l];
  if (tid < M) {
    sh.xb[0][tid][0] = sh.px[tid * M];
    sh.xb[1][tid][0] = sh.px[tid * M + M - 1];
    sh.xb[2][tid][0] = sh.px[tid];
    sh.xb[3][tid][0] = sh.px[(M - 1) * M + tid];
  }
  __syncthreads();
  write_block(a, sd, I, J, sh.fc, sh.xb);
}

// One wavefront per SIMD: the FP32 inverse blocks live beside the FP64
// solution, residual and correction tiles, which at two wavefronts per SIMD
// (256 registers) spilled 103 dwords per lane to scratch; at one the
// compiler keeps them in the accumulation registers instead (local phase
// 0.72 -> 0.58 ms at 1024^2).
__global__ void __launch_bounds__(PAIR, 1) basis32_pair_kernel(SubArgs a) {
  __shared__ Lds32 sh;
  if (__builtin_amdgcn_readfirstlane(threadIdx.x >> 6) == 0) basis32_body<0>(a, sh);
  else basis32_body<1>(a, sh);
}

// ---------------------------------------------------------------------------
// stitch re-solve for 16 x 16 subdomains (two wavefronts per subdomain)
// ---------------------------------------------------------------------------

// interface coefficient of basis column q of subdomain (I, J) (0 for a side
// on the domain boundary, whose basis columns are zero)
template <int DD = D>
__device__ inline double column_coef(const SubArgs& a, int I, int J, int q) {
  const int e = side_iface(a.g, I, J, q / DD);
  return e >= 0 ? a.coef[(size_t)e * DD + q % DD] : 0.0;
}

// composed pressure p = X [1; c] at cell l of subdomain sd, coefficients cf
// of its 4 DD basis columns; the loads are issued 16 at a time, unconditionally
template <int DD>
__device__ inline double compose(const SubArgs& a, int sd, int l, const double* cf) {
  const double* xr = a.X + (size_t)sd * (4 * DD + 1) * MM + l;
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

// The composed pressure p = X [1; c] of every cell (the multiscale solution
// from the local solutions and the interface coefficients; it is the
// pressure output) and each subdomain's pressure sum (for the zero-mean
// shift without Dirichlet data), one work-group per subdomain, two
// neighbouring cells per thread (16-byte loads, each cell's sum in the
// order of compose): a streaming pass over X, so that the stitch kernel,
// whose work is the latency-bound re-solve, reads only the pressures next
// to its faces.
constexpr int COMPOSE_NT = MM / 2;
template <int DD>
__global__ void __launch_bounds__(COMPOSE_NT) compose_kernel(SubArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) stamp_now(a.stamps + STAMP_FLUX);
  __shared__ double cfs[4 * DD];
  __shared__ double red[COMPOSE_NT / WAVE];
  const Geo& g = a.g;
  const int sd = blockIdx.x, t = threadIdx.x, l = 2 * t;
  const int I = sd % g.SX, J = sd / g.SX;
  if (t < 4 * DD) cfs[t] = column_coef<DD>(a, I, J, t);
  __syncthreads();
  typedef double dbl2 __attribute__((ext_vector_type(2)));
  const dbl2* xr = reinterpret_cast<const dbl2*>(a.X + (size_t)sd * (4 * DD + 1) * MM + l);
  dbl2 p = __builtin_nontemporal_load(xr);
#pragma unroll
  for (int q0 = 0; q0 < 4 * DD; q0 += 16) {
    dbl2 x[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) x[q] = __builtin_nontemporal_load(xr + (size_t)(1 + q0 + q) * (MM / 2));
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      p.x = fma(x[q].x, cfs[q0 + q], p.x);
      p.y = fma(x[q].y, cfs[q0 + q], p.y);
    }
  }
  double* po = a.p_out + (size_t)(J * M + l / M) * g.nx + I * M + l % M;
  po[0] = p.x;
  po[1] = p.y;
  double s = p.x + p.y;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((t & (WAVE - 1)) == 0) red[t / WAVE] = s;
  __syncthreads();
  if (t == 0) {
    double u = red[0];
#pragma unroll
    for (int k = 1; k < COMPOSE_NT / WAVE; ++k) u += red[k];
    a.sub_stats[3 * sd + 2] = u;
  }
}

// a register budget of two wavefronts per SIMD: 155 registers per lane, no
// spills, so three wavefronts fit (19 KB of LDS per pair); the flux phase is
// about 8 us shorter at 1024^2 than at four wavefronts per SIMD with 128
// registers and 84 bytes of spills per lane
template <int DD>
__global__ void __launch_bounds__(PAIR, 2) stitch_pair_kernel(SubArgs a) {
  __shared__ double kap[MM], dg[MM], ex[MM], cy[MM];
  __shared__ double bs_[MM], ps[MM], rs[MM];
  __shared__ double pm0;   // composed pressure of cell 0 (the pin)
  __shared__ double Fout[4][M];
  __shared__ double red[2][2];
  __shared__ double xch[M][M + 1];
  const Geo& g = a.g;
  // the wave index is uniform per wavefront: taken into a scalar register,
  // so that row offsets that depend on it are scalar too
  const int tid = threadIdx.x, w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int lane = tid & 63, c = lane & 15, gq = lane >> 4;
  // Consecutive subdomains on one XCD: work-groups go to the 8 XCDs in
  // turn, so work-group b takes subdomain (b mod 8) n/8 + b/8, and the
  // lines of the neighbours' face cells that a work-group reads were mostly
  // loaded into the same L2 by the neighbours' own work-groups.
  const int nbk = gridDim.x;
  const int sd = (nbk % 8 == 0) ? (blockIdx.x % 8) * (nbk / 8) + blockIdx.x / 8 : blockIdx.x;
  const int I = sd % g.SX, J = sd / g.SX;
  const int nP = g.nP;

  // both sides of each skeleton face (first 4 M threads): the composed
  // pressures next to the face (written by compose_kernel) and the
  // neighbour's mobility
  const int side = lane >> 4, t = lane & 15;
  const int e = tid < 4 * M ? side_iface(g, I, J, side) : -1;
  double pn = 0.0, po = 0.0, kn = 1.0, al = 0.0, PH = 0.0, UH = 0.0;
  size_t nc_g = 0;   // the neighbour's cell (global index)
  if (tid == 0) pm0 = a.p_out[(size_t)(J * M) * g.nx + I * M];
  if (e >= 0) {
    // interface data of the face: alpha and the interface pressure / flux
    // P_H, U_H = sum of coefficient times interface function
    al = a.alpha[e];
    const double* bsf = a.basis + (size_t)e * DD * M;
    const double* ce = a.coef + (size_t)e * DD;
    for (int k = 0; k < nP; ++k) PH += ce[k] * bsf[k * M + t];
    for (int k = nP; k < DD; ++k) UH += ce[k] * bsf[k * M + t];
    const int nside = side ^ 1;
    const int nsd = (side == 0) ? sd - 1 : (side == 1) ? sd + 1 : (side == 2) ? sd - g.SX : sd + g.SX;
    const int nI = nsd % g.SX, nJ = nsd / g.SX;
    const int nl = side_cell<M>(nside, t);
    const size_t nc = (size_t)(nJ * M + nl / M) * g.nx + nI * M + nl % M;
    nc_g = nc;
    kn = a.K[nc] * a.lam[nc];
    pn = a.p_out[nc];
    const int lo = side_cell<M>(side, t);
    po = a.p_out[(size_t)(J * M + lo / M) * g.nx + I * M + lo % M];
  }
  CellLoads cl[MM / PAIR];   // issued with the permeability loads
#pragma unroll
  for (int q = 0; q < MM / PAIR; ++q) cl[q] = cell_loads<M>(a, I, J, tid + PAIR * q, 0);
  load_kappa<M>(a, I, J, kap);
  __syncthreads();
  if (tid < 4 * M) {
    // one-sided Robin fluxes on both sides of each skeleton face; outflow
    // of this subdomain = their average
    double fo = 0.0;
    if (e >= 0) {
      const SideGeo sg = side_geo(g, side);
      const int l = side_cell<M>(side, t);
      const double sig = side_sigma(side);
      const double ko = kap[l];
      const double TRo = sg.flen * ko / (sg.dist + al * sg.H), TRn = sg.flen * kn / (sg.dist + al * sg.H);
      double Fown = TRo * (po - (PH - al * sg.H / ko * sig * UH));
      double Fnb = TRn * (pn - (PH - al * sg.H / kn * (-sig) * UH));
      if (a.rho) {
        Fown += robin_grav(a, side, (size_t)(J * M + l / M) * g.nx + I * M + l % M, TRo, sg.dist);
        Fnb += robin_grav(a, side ^ 1, nc_g, TRn, sg.dist);
      }
      fo = 0.5 * (Fown - Fnb);
    }
    Fout[side][t] = fo;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MM / PAIR; ++q)
    assemble_cell<M, 1, false>(a, I, J, tid + PAIR * q, kap, dg, ex, cy, bs_ + tid + PAIR * q, 0, Fout,
                               cl[q]);
  __syncthreads();
  const bool dir = (I == 0 && g.kind[0] == 1) || (I == g.SX - 1 && g.kind[1] == 1) ||
                   (J == 0 && g.kind[2] == 1) || (J == g.SY - 1 && g.kind[3] == 1);
  // A subdomain with no Dirichlet face has a Neumann problem, solvable only
  // if its data sum to zero.  The averaged skeleton fluxes meet this to the
  // rounding of the composed solution; that defect (summed in double-double)
  // is removed evenly from the cells' data instead of being left to the
  // pinned cell, and the constant is fixed at cell 0 to the composed
  // pressure (its pin then carries no flux).
  // per-cell defect share and pin transmissibility, kept in LDS across the
  // factorisation (in registers they would push its inverse blocks out)
  __shared__ double pin_sc[2];
  if (tid == 0) {
    pin_sc[0] = 0.0;
    pin_sc[1] = 0.0;
  }
  if (!dir) {   // uniform over the work-group
    double sh = 0.0, sl = 0.0;
#pragma unroll
    for (int q = 0; q < MM / PAIR; ++q) dd_add(sh, sl, bs_[tid + PAIR * q]);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
      const double oh = __shfl_xor(sh, off), ol = __shfl_xor(sl, off);
      dd_add(sh, sl, oh);
      sl += ol;
    }
    if (lane == 0) {
      red[0][w] = sh;
      red[1][w] = sl;
    }
    __syncthreads();
    sh = red[0][0];
    sl = red[1][0];
    dd_add(sh, sl, red[0][1]);
    sl += red[1][1];
    const double dfc = (sh + sl) / MM;
#pragma unroll
    for (int q = 0; q < MM / PAIR; ++q) bs_[tid + PAIR * q] -= dfc;
    if (tid == 0) {    // thread 0 owns cell 0
      const double tp = dg[0];
      dg[0] += tp;
      bs_[0] += tp * pm0;
      pin_sc[0] = dfc;
      pin_sc[1] = tp;
    }
  }
  __syncthreads();

  d4 Sv[NU];
  PivotCheck pvc;
  factor_pair<DD>(Sv, w, c, gq, dg, ex, cy, xch, pvc);
  if (pvc.bad()) atomicOr(a.status, ST_STITCH_PIVOT);
  solve_column_pair<DD>(Sv, w, bs_, ps, c, gq, cy);
  // one step of iterative refinement with the stored inverse blocks; the
  // residual is the cells' mass balance in double-double (the FP64 diagonal
  // sums of the assembled matrix would leave eps * T |p| per cell), and the
  // pressure is kept as the unevaluated sum ps + rs (solution + correction)
  // from which the fluxes are formed: the cell balances then hold to the
  // rounding of the fluxes themselves
#pragma unroll 1
  for (int q = 0; q < MM / PAIR; ++q) {   // one cell at a time: the inverse blocks stay in registers
    const int l = tid + PAIR * q;
    rs[l] = stitch_balance_residual<M>(a, I, J, l, kap, ps, Fout, pin_sc[0], pin_sc[1], pm0);
  }
  __syncthreads();
  solve_column_pair<DD>(Sv, w, rs, rs, c, gq, cy);   // in place: each row is read before it is written

  double imb = 0.0, fmx = 0.0;
#pragma unroll 1
  for (int l = tid; l < MM; l += PAIR) {
    const int li = l % M, lj = l / M;
    const int i = I * M + li, j = J * M + lj;
    double out[4];
    stitch_out_fluxes<M>(a, I, J, l, kap, ps, rs, Fout, out);
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
  }
  // reductions over the wave (fixed butterfly order), then over the two waves
  // (the pressure sum of the subdomain is compose_kernel's)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    imb = fmax(imb, __shfl_xor(imb, off));
    fmx = fmax(fmx, __shfl_xor(fmx, off));
  }
  if (lane == 0) {
    red[0][w] = imb;
    red[1][w] = fmx;
  }
  __syncthreads();
  if (tid == 0) {
    a.sub_stats[3 * sd + 0] = fmax(red[0][0], red[0][1]);
    a.sub_stats[3 * sd + 1] = fmax(red[1][0], red[1][1]);
  }
}

// ---------------------------------------------------------------------------
// learned surrogate of the 16 basis functions: network inputs, training
// targets and the FP64 residual gate (the network itself is in surrogate.hip)
// ---------------------------------------------------------------------------

__device__ inline short to_bf16(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (short)(u >> 16);
}

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  return v;
}

// mean of ln kappa over the subdomain (every lane gets it)
__device__ inline double mean_log_kappa(const double* kap) {
  double s = 0.0;
  for (int l = threadIdx.x; l < MM; l += WAVE) s += log(kap[l]);
  return wave_sum(s) / MM;
}

// normalisation of network output column q (dof k of side q/4): 1 for
// pressure dofs, kappa_g / (alpha H) for flux dofs, 0 where the side lies on
// the domain boundary (that column is identically zero)
__device__ inline double column_scale(const SubArgs& a, int I, int J, int q, double kgeo) {
  const int side = q / D, k = q % D;
  const int e = side_iface(a.g, I, J, side);
  if (e < 0) return 0.0;
  if (k < a.g.nP) return 1.0;
  return kgeo / (a.alpha[e] * side_geo(a.g, side).H);
}

__global__ void __launch_bounds__(WAVE) surrogate_inputs_kernel(SubArgs a, short* inputs) {
  __shared__ double kap[MM];
  const Geo& g = a.g;
  const int sd = blockIdx.x, I = sd % g.SX, J = sd / g.SX;
  load_kappa<M>(a, I, J, kap);
  __syncthreads();
  const double mean = mean_log_kappa(kap);
  bool has[4];
  for (int side = 0; side < 4; ++side) has[side] = side_iface(g, I, J, side) >= 0;
  short* out = inputs + (size_t)sd * MM * 8;
  for (int l = threadIdx.x; l < MM; l += WAVE) {
    const int li = l % M, lj = l / M;
    typedef short s8 __attribute__((ext_vector_type(8)));
    s8 v = {0, 0, 0, 0, 0, 0, 0, 0};
    const short one = to_bf16(1.f);
    v[0] = to_bf16((float)((log(kap[l]) - mean) * 0.25));
    if (has[0] && li == 0) v[1] = one;
    if (has[1] && li == M - 1) v[2] = one;
    if (has[2] && lj == 0) v[3] = one;
    if (has[3] && lj == M - 1) v[4] = one;
    *reinterpret_cast<s8*>(out + (size_t)l * 8) = v;
  }
}

__global__ void __launch_bounds__(WAVE) surrogate_targets_kernel(SubArgs a, float* targets) {
  __shared__ double kap[MM];
  __shared__ double scale[4 * D];
  const Geo& g = a.g;
  const int sd = blockIdx.x, I = sd % g.SX, J = sd / g.SX;
  load_kappa<M>(a, I, J, kap);
  __syncthreads();
  const double kgeo = exp(mean_log_kappa(kap));
  if (threadIdx.x < 4 * D) scale[threadIdx.x] = column_scale(a, I, J, threadIdx.x, kgeo);
  __syncthreads();
  const double* Xg = a.X + (size_t)sd * R * MM;
  float* out = targets + (size_t)sd * MM * 4 * D;
  for (int o = threadIdx.x; o < MM * 4 * D; o += WAVE) {
    const int l = o / (4 * D), q = o % (4 * D);
    out[o] = (float)(Xg[(size_t)(1 + q) * MM + l] * scale[q]);
  }
}

// Decode the network's prediction of the 16 basis functions, smooth them
// with a few FP64 red-black Gauss-Seidel sweeps of the local Robin problem,
// form each column's FP64 residual and accept the subdomain only if every
// column passes; an accepted subdomain gets its basis block
// and its block of the interface system written exactly as the FP64 kernel
// would, a rejected one (or one with source or physical boundary data,
// whose particular solution the network does not predict) is appended to
// a.fallback for the FP64 kernel.
constexpr int GATE = 256;   // threads of the gate kernel: one per cell
constexpr int GATE_SWEEPS = 4;   // red-black Gauss-Seidel sweeps before the gate

__global__ void __launch_bounds__(GATE) surrogate_gate_kernel(SubArgs a, const float* pred) {
  __shared__ double kap[MM], dg[MM], ex[MM], cy[MM], b0[MM];
  __shared__ double bside[4][M][D];
  __shared__ Faces fc;
  __shared__ double xb[4][M][R];
  __shared__ double Xs[4 * D][MM];        // decoded basis functions
  __shared__ double scale[4 * D];
  __shared__ double part[GATE / WAVE][2][4 * D];
  __shared__ int verdict;
  const Geo& g = a.g;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int sd = blockIdx.x, I = sd % g.SX, J = sd / g.SX;
  static_assert(GATE == MM, "one thread per cell");

  const FaceLoadT<D> fl = load_faces(a, I, J);
  const float* pr = pred + (size_t)sd * MM * 4 * D;
  // raw predictions, cell-major in memory: 16 per thread, coalesced (entry
  // tid + k GATE is column tid % 16 of cell tid / 16 + 16 k)
  float praw[4 * D];
#pragma unroll
  for (int k = 0; k < 4 * D; ++k) praw[k] = pr[tid + k * GATE];
  const CellLoads cl = cell_loads<M>(a, I, J, tid, 1);   // issued with the permeability loads
  load_kappa<M>(a, I, J, kap);
  __syncthreads();
  assemble_cell<M, 1, false>(a, I, J, tid, kap, dg, ex, cy, b0 + tid, 1, nullptr, cl);
  if (wv == 0) {
    // the same geometric mean (same summation order) as the input and
    // target builders
    const double kgeo = exp(mean_log_kappa(kap));
    if (lane < 4 * D) scale[lane] = column_scale(a, I, J, lane, kgeo);
  }
  prepare_faces(a, fl, kap, fc, I, J);
  __syncthreads();
  robin_data(g, fc, bside);
  {
    const int q = tid % (4 * D);
    const double sc = scale[q];
#pragma unroll
    for (int k = 0; k < 4 * D; ++k) Xs[q][tid / (4 * D) + k * (GATE / (4 * D))] = sc != 0.0 ? (double)praw[k] / sc : 0.0;
  }
  const int particular = __syncthreads_or(b0[tid] != 0.0);

  // residual of every column at cell tid, squared norms per column
  const int i = tid % M, j = tid / M;
  const int le = i < M - 1 ? tid + 1 : tid, lw = i > 0 ? tid - 1 : tid;
  const int ln = j < M - 1 ? tid + M : tid, ls = j > 0 ? tid - M : tid;
  const double ce = i < M - 1 ? ex[tid] : 0.0, cw = i > 0 ? ex[lw] : 0.0;
  const double cn = j < M - 1 ? cy[tid] : 0.0, cs = j > 0 ? cy[ls] : 0.0;
  // The network's output is FP32: rounding an exact basis function to FP32
  // alone leaves a relative residual of about 2e-6 (spread over all cells,
  // while b lives on the boundary cells), above a 1e-6 gate.  A few
  // red-black Gauss-Seidel sweeps in FP64 remove that rounding noise (it is
  // high-frequency, which point relaxation damps fastest) before the gate
  // measures the residual; they need no factorisation, and what they cannot
  // correct (an approximation error of the network, smooth over the
  // subdomain) still fails the gate.
  {
    const double idg = 1.0 / dg[tid];
    const int color = (i + j) & 1;
#pragma unroll 1
    for (int half = 0; half < 2 * GATE_SWEEPS; ++half) {
      if (color == (half & 1)) {   // a colour's neighbours all have the other colour
#pragma unroll
        for (int q = 0; q < 4 * D; ++q) {
          double ax = dg[tid] * Xs[q][tid];
          ax = fma(ce, Xs[q][le], ax);
          ax = fma(cw, Xs[q][lw], ax);
          ax = fma(cn, Xs[q][ln], ax);
          ax = fma(cs, Xs[q][ls], ax);
          Xs[q][tid] += (side_rhs(bside, j, i, q) - ax) * idg;
        }
      }
      __syncthreads();
    }
  }
  double r2[4 * D], b2[4 * D];
#pragma unroll
  for (int q = 0; q < 4 * D; ++q) {
    double ax = dg[tid] * Xs[q][tid];
    ax = fma(ce, Xs[q][le], ax);
    ax = fma(cw, Xs[q][lw], ax);
    ax = fma(cn, Xs[q][ln], ax);
    ax = fma(cs, Xs[q][ls], ax);
    const double bq = side_rhs(bside, j, i, q);
    const double r = bq - ax;
    r2[q] = wave_sum(r * r);
    b2[q] = wave_sum(bq * bq);
  }
  if (lane == 0) {
#pragma unroll
    for (int q = 0; q < 4 * D; ++q) {
      part[wv][0][q] = r2[q];
      part[wv][1][q] = b2[q];
    }
  }
  __syncthreads();
  if (tid < WAVE) {
    bool ok = true;
    if (tid < 4 * D) {
      double rr = 0.0, bb = 0.0;
      for (int w = 0; w < GATE / WAVE; ++w) {
        rr += part[w][0][tid];
        bb += part[w][1][tid];
      }
      ok = isfinite(rr) && rr <= a.gate_tol * a.gate_tol * bb;
    }
    const bool accept = __all(ok) && !particular;
    if (tid == 0) {
      verdict = accept;
      if (!accept) {
        const int q = atomicAdd(a.fallback, 1);
        a.fallback[1 + q] = sd;
      }
    }
  }
  __syncthreads();
  if (!verdict) return;

  // accepted: the decoded basis block and the interface block
  double* Xg = a.X + (size_t)sd * R * MM;
  Xg[tid] = 0.0;   // no particular data
#pragma unroll
  for (int q = 0; q < 4 * D; ++q) Xg[(size_t)(1 + q) * MM + tid] = Xs[q][tid];
  for (int o = tid; o < 4 * M * R; o += GATE) {
    const int side = o / (M * R), t = (o / R) % M, col = o % R;
    double v = 0.0;
    if (col > 0) {
      const int l = side_cell<M>(side, t);
      v = Xs[col - 1][l];
    }
    xb[side][t][col] = v;
  }
  __syncthreads();
  write_block(a, sd, I, J, fc, xb);
}

}  // namespace

hipError_t launch_basis_m16d4(const SubArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((basis_pair_kernel<false, 4>), dim3(a.g.n_sub), dim3(PAIR), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_basis_m16d4_list(const SubArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((basis_pair_kernel<true, 4>), dim3(a.g.n_sub), dim3(PAIR), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_basis_m16d8(const SubArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((basis_pair_kernel<false, 8>), dim3(2 * a.g.n_sub), dim3(PAIR), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_basis32_m16d4(const SubArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(basis32_pair_kernel, dim3(a.g.n_sub), dim3(PAIR), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_stitch_m16d4(const SubArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(compose_kernel<4>, dim3(a.g.n_sub), dim3(COMPOSE_NT), 0, st, a);
  hipLaunchKernelGGL(stitch_pair_kernel<4>, dim3(a.g.n_sub), dim3(PAIR), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_stitch_m16d8(const SubArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(compose_kernel<8>, dim3(a.g.n_sub), dim3(COMPOSE_NT), 0, st, a);
  hipLaunchKernelGGL(stitch_pair_kernel<8>, dim3(a.g.n_sub), dim3(PAIR), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_surrogate_inputs(const SubArgs& a, short* inputs, hipStream_t st) {
  hipLaunchKernelGGL(surrogate_inputs_kernel, dim3(a.g.n_sub), dim3(WAVE), 0, st, a, inputs);
  return hipGetLastError();
}

hipError_t launch_surrogate_targets(const SubArgs& a, float* targets, hipStream_t st) {
  hipLaunchKernelGGL(surrogate_targets_kernel, dim3(a.g.n_sub), dim3(WAVE), 0, st, a, targets);
  return hipGetLastError();
}

hipError_t launch_surrogate_gate(const SubArgs& a, const float* pred, hipStream_t st) {
  hipLaunchKernelGGL(surrogate_gate_kernel, dim3(a.g.n_sub), dim3(GATE), 0, st, a, pred);
  return hipGetLastError();
}

}  // namespace mrcm
