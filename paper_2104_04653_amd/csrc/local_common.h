// Device helpers shared by the per-subdomain kernels: geometry of the
// subdomain sides and the assembly of one cell of the local two-point
// system (paper, section 3: eq. (mrc1) with the Robin parameter of eq.
// (beta); physical Dirichlet/Neumann data of eq. (Darcy)).
#pragma once

#include "mrcm_internal.h"

#include <math.h>

namespace mrcm {
namespace local {

// transmissibility of a face from the half-cell transmissibilities of its
// two cells (in series): one division, and symmetric in a and b, so both
// cells of a face compute the same value
__device__ inline double series2(double a, double b) { return a * b / (a + b); }

// (hi, lo) += b with an error-free two-sum
__device__ inline void dd_add(double& hi, double& lo, double b) {
#pragma clang fp contract(off)
  const double s = hi + b;
  const double bb = s - hi;
  lo += (hi - (s - bb)) + (b - bb);
  hi = s;
}


struct SideGeo {
  double flen, dist, H;
};

__device__ inline SideGeo side_geo(const Geo& g, int side) {
  SideGeo s;
  if (side < 2) {
    s.flen = g.hy; s.dist = 0.5 * g.hx; s.H = g.M * g.hy;
  } else {
    s.flen = g.hx; s.dist = 0.5 * g.hy; s.H = g.M * g.hx;
  }
  return s;
}

// interface on side (W,E,S,N) of subdomain (I,J), -1 on the domain boundary
__device__ inline int side_iface(const Geo& g, int I, int J, int side) {
  switch (side) {
    case 0: return I > 0 ? J * (g.SX - 1) + I - 1 : -1;
    case 1: return I < g.SX - 1 ? J * (g.SX - 1) + I : -1;
    case 2: return J > 0 ? g.nV + (J - 1) * g.SX + I : -1;
    default: return J < g.SY - 1 ? g.nV + J * g.SX + I : -1;
  }
}

// n . n_i: +1 where the subdomain is the lower-index side (E and N sides)
__device__ inline double side_sigma(int side) { return (side == 1 || side == 3) ? 1.0 : -1.0; }

// local cell index of face t on a side
template <int M>
__device__ inline int side_cell(int side, int t) {
  switch (side) {
    case 0: return t * M;
    case 1: return t * M + (M - 1);
    case 2: return t;
    default: return (M - 1) * M + t;
  }
}

// The global values one cell's assembly reads: the source, and per side the
// boundary value (domain boundary) and the Robin parameter (skeleton).
struct CellLoads {
  double sv, bv[4], av[4];
  double rc, rs, rn;      // gravity: lambda_g / lambda of the cell and its S, N neighbours
};

// Gravity (section 5.5: u = -kappa (grad p - rho gamma e_y), rho =
// lambda_g / lambda per cell, gamma = g dh/dy): the constant part of the
// flux out of a cell through one of its faces, T gamma d rho for a half
// cell of transmissibility T and centre-to-face distance d (a face between
// two cells: T their series transmissibility, d h/2 and rho the sum of the
// two cells' values), signed by the face's outward normal (+1 on N, -1 on
// S, 0 on the x-faces).
__device__ inline double grav_out(const Geo& g, int side, double T, double d, double rho) {
  return side < 2 ? 0.0 : (side == 3 ? 1.0 : -1.0) * T * g.grav * d * rho;
}

// physics spaces: slot k of interface e holds a function (pressure slots
// 0 .. nP-1, flux slots nP .. D-1, the first nact[e] of each in use)
__device__ inline bool slot_active(const SubArgs& a, int e, int k) {
  const int2 n = a.nact[e];
  return k < a.g.nP ? k < n.x : k - a.g.nP < n.y;
}

// the gravity part of the one-sided Robin flux out of cell c (global index)
// through `side`: T_R gamma d rho_c (n . e_y); zero without gravity
__device__ inline double robin_grav(const SubArgs& a, int side, size_t c, double TR, double d) {
  return a.rho ? grav_out(a.g, side, TR, d, a.rho[c]) : 0.0;
}

// Loaded without branches, each from an address selected per side (the
// cell's own permeability stands in where the value is not needed), so that
// a thread's loads are all in flight together: loads behind branches wait
// one by one.
template <int M>
__device__ inline CellLoads cell_loads(const SubArgs& a, int I, int J, int l, int robin) {
  const Geo& g = a.g;
  const int li = l % M, lj = l / M;
  const int i = I * M + li, j = J * M + lj;
  const size_t c = (size_t)j * g.nx + i;
  const double* stand = a.K + c;
  CellLoads cl;
  cl.sv = *(a.src ? a.src + c : stand);
#pragma unroll
  for (int side = 0; side < 4; ++side) {
    const bool inner = (side == 0) ? li > 0 : (side == 1) ? li < M - 1 : (side == 2) ? lj > 0 : lj < M - 1;
    const int e = inner ? 0 : side_iface(g, I, J, side);
    cl.bv[side] = *((!inner && e < 0) ? a.bcv[side] + ((side < 2) ? j : i) : stand);
    cl.av[side] = *((!inner && e >= 0 && robin) ? a.alpha + e : stand);
  }
  cl.rc = cl.rs = cl.rn = 0.0;
  if (a.rho) {
    cl.rc = a.rho[c];
    cl.rs = a.rho[lj > 0 ? c - g.nx : c];
    cl.rn = a.rho[lj < M - 1 ? c + g.nx : c];
  }
  return cl;
}

// Assemble one cell of the local two-point system: diagonal, coupling to the
// +x neighbour (ex) and to the +y neighbour (cy), and the cell's row of the
// right-hand sides.  robin != 0: skeleton faces carry the Robin law (the
// basis-function problems); robin == 0: skeleton faces carry the prescribed
// outflow Fout[side][t] (the stitch re-solve).  cl: the cell's values from
// cell_loads (a kernel may load several cells' values before assembling).
template <int M, int R, bool SIDES = true>
__device__ void assemble_cell(const SubArgs& a, int I, int J, int l, const double* kap,
                              double* dg, double* ex, double* cy, double* xrow, int robin,
                              const double (*Fout)[M], const CellLoads& cl, float* dgl = nullptr) {
  const Geo& g = a.g;
  const int li = l % M, lj = l / M;
  const int i = I * M + li, j = J * M + lj;
  const double kc = kap[l];
  const double txc = kc * g.tfx;
  const double tyc = kc * g.tfy;
  // the diagonal is a sum of transmissibilities; its FP64 rounding error
  // (dlo, kept with an error-free two-sum) makes (diag + dlo) x exactly the
  // flux form sum of T (x_c - x_nb), so that residuals formed with it are the
  // cells' mass balances (a rounded diagonal leaves eps T |x| per cell, which
  // sums to a conservation defect of the local solutions)
  double diag = 0.0, dlo = 0.0, cx = 0.0, cn = 0.0;
  for (int q = 0; q < R; ++q) xrow[q] = 0.0;
  double rhs0 = 0.0;
  if (a.src) rhs0 += cl.sv * g.hx * g.hy;
  // face loop: side 0 W, 1 E, 2 S, 3 N
#pragma unroll
  for (int side = 0; side < 4; ++side) {
    const bool inner = (side == 0) ? li > 0 : (side == 1) ? li < M - 1 : (side == 2) ? lj > 0 : lj < M - 1;
    if (inner) {
      int nb = (side == 0) ? l - 1 : (side == 1) ? l + 1 : (side == 2) ? l - M : l + M;
      double tn = kap[nb] * ((side < 2) ? g.tfx : g.tfy);
      double T = series2(side < 2 ? txc : tyc, tn);
      dd_add(diag, dlo, T);
      if (side == 1) cx = -T;
      if (side == 3) cn = -T;
      if (a.rho) rhs0 -= grav_out(g, side, T, 0.5 * g.hy, cl.rc + (side == 2 ? cl.rs : cl.rn));
      continue;
    }
    const int e = side_iface(g, I, J, side);
    const int t = (side < 2) ? lj : li;
    const double th = (side < 2) ? txc : tyc;
    if (e < 0) {  // physical boundary
      const double flen = (side < 2) ? g.hy : g.hx;
      const double v = cl.bv[side];
      if (g.kind[side] == 1) {
        dd_add(diag, dlo, th);
        rhs0 += th * v;
        if (a.rho) rhs0 -= grav_out(g, side, th, 0.5 * g.hy, cl.rc);
      } else {
        rhs0 -= v * flen;
      }
      continue;
    }
    if (robin) {
      SideGeo sg = side_geo(g, side);
      const double al = cl.av[side];
      const double TR = sg.flen * kc / (sg.dist + al * sg.H);
      const double beta = al * sg.H / kc;
      const double sig = side_sigma(side);
      dd_add(diag, dlo, TR);
      // gravity through the Robin face: data of the particular solution
      if (a.rho) rhs0 -= grav_out(g, side, TR, sg.dist, cl.rc);
      if (SIDES) {
        const int D = g.D;
        const double* bs = a.basis + (size_t)e * D * M;
        for (int k = 0; k < D; ++k) {
          double gv = bs[k * M + t];
          if (k >= g.nP) gv = -beta * sig * gv;
          xrow[1 + side * D + k] += TR * gv;
        }
      }
    } else {
      rhs0 -= Fout[side][t];
    }
  }
  dg[l] = diag;
  if (dgl) dgl[l] = (float)dlo;
  ex[l] = cx;
  cy[l] = cn;
  xrow[0] += rhs0;
}

// the same, loading the cell's values itself
template <int M, int R, bool SIDES = true>
__device__ void assemble_cell(const SubArgs& a, int I, int J, int l, const double* kap,
                              double* dg, double* ex, double* cy, double* xrow, int robin,
                              const double (*Fout)[M], float* dgl = nullptr) {
  assemble_cell<M, R, SIDES>(a, I, J, l, kap, dg, ex, cy, xrow, robin, Fout,
                             cell_loads<M>(a, I, J, l, robin), dgl);
}

// (hi, lo) += a * b in double-double arithmetic: the product is split
// exactly with an FMA and added with an error-free two-sum, so a residual
// b - A x accumulated this way carries about twice the FP64 precision
// (used by the iterative refinement of the local solves).
__device__ inline void dd_fma(double& hi, double& lo, double a, double b) {
#pragma clang fp contract(off)
  const double p = a * b;
  const double pe = fma(a, b, -p);
  const double s = hi + p;
  const double bb = s - hi;
  const double se = (hi - (s - bb)) + (p - bb);
  hi = s;
  lo += pe + se;
}

// (hi, lo) += a b for a product at most eps |hi| (the rounding error of a
// diagonal sum times the solution): it goes into the low part alone, whose
// own rounding error is then of order eps^2 |hi|, as dd_fma's
__device__ inline void dd_fma_low(double& lo, double a, double b) { lo = fma(a, b, lo); }

// (ah + al) - (bh + bl) rounded once to FP64: the difference of the leading
// parts is taken with an error-free two-difference, so a face flux
// T ((p_c - p_d)) formed from pressures carried as unevaluated sums keeps
// its relative accuracy when the two pressures nearly cancel (the stitched
// cell balances then hold to rounding of the fluxes themselves, not of the
// pressures).
__device__ inline double dd_diff(double ah, double al, double bh, double bl) {
#pragma clang fp contract(off)
  const double s = ah - bh;
  const double v = s - ah;
  const double e = (ah - (s - v)) + (-bh - v);
  return s + (e + (al - bl));
}

// Outward fluxes of cell l through its W, E, S, N faces in the stitch
// re-solve, from the pressure ph + pl (pl may be NULL): the two-point law
// inside the subdomain, the prescribed averaged flux Fout on skeleton faces,
// the physical law on the domain boundary (Dirichlet t_c (p - p_b), Neumann
// u_b |f|).  The same expressions form the residual of the re-solve and its
// output fluxes, so the refined pressure balances the fluxes it outputs.
template <int M>
__device__ inline void stitch_out_fluxes(const SubArgs& a, int I, int J, int l, const double* kap,
                                         const double* ph, const double* pl,
                                         const double (*Fout)[M], double out[4]) {
  const Geo& g = a.g;
  const int li = l % M, lj = l / M;
  const int i = I * M + li, j = J * M + lj;
  const double kc = kap[l];
  const double txc = kc * g.tfx, tyc = kc * g.tfy;
  const double pv = ph[l], pvl = pl ? pl[l] : 0.0;
#pragma unroll
  for (int side = 0; side < 4; ++side) {
    const bool inner = (side == 0) ? li > 0 : (side == 1) ? li < M - 1 : (side == 2) ? lj > 0 : lj < M - 1;
    if (inner) {
      const int nb = (side == 0) ? l - 1 : (side == 1) ? l + 1 : (side == 2) ? l - M : l + M;
      const double tn = kap[nb] * ((side < 2) ? g.tfx : g.tfy);
      const double T = series2(side < 2 ? txc : tyc, tn);
      out[side] = T * dd_diff(pv, pvl, ph[nb], pl ? pl[nb] : 0.0);
      if (a.rho && side >= 2) {
        const size_t c = (size_t)j * g.nx + i;
        out[side] += grav_out(g, side, T, 0.5 * g.hy, a.rho[c] + a.rho[side == 2 ? c - g.nx : c + g.nx]);
      }
    } else {
      const int e = side_iface(g, I, J, side);
      const int t = (side < 2) ? lj : li;
      if (e >= 0) {
        out[side] = Fout[side][t];
      } else {
        const double flen = (side < 2) ? g.hy : g.hx;
        const double v = a.bcv[side][(side < 2) ? j : i];
        out[side] = (g.kind[side] == 1) ? ((side < 2) ? txc : tyc) * dd_diff(pv, pvl, v, 0.0) : v * flen;
        if (a.rho && g.kind[side] == 1) out[side] += grav_out(g, side, tyc, 0.5 * g.hy, a.rho[(size_t)j * g.nx + i]);
      }
    }
  }
}

// Residual of cell l of the stitch re-solve written as its mass balance,
// q |V| - dfc - (net outflow) - (pin flux of a floating subdomain's cell 0),
// in double-double from the pressure ph (FP64); dfc is the per-cell share
// of the Neumann data's compatibility defect, tp the pin transmissibility
// and pref the pinned value (tp = 0: no pin).
template <int M>
__device__ inline double stitch_balance_residual(const SubArgs& a, int I, int J, int l,
                                                 const double* kap, const double* ph,
                                                 const double (*Fout)[M], double dfc, double tp,
                                                 double pref) {
  const Geo& g = a.g;
  const int li = l % M, lj = l / M;
  const int i = I * M + li, j = J * M + lj;
  const double kc = kap[l], pv = ph[l];
  double hi = a.src ? a.src[(size_t)j * g.nx + i] * g.hx * g.hy : 0.0, lo = 0.0;
  dd_add(hi, lo, -dfc);
  // the faces one at a time (the caller keeps its inverse blocks in
  // registers meanwhile); the same face laws as stitch_out_fluxes
#pragma unroll 1
  for (int side = 0; side < 4; ++side) {
    const bool inner = (side == 0) ? li > 0 : (side == 1) ? li < M - 1 : (side == 2) ? lj > 0 : lj < M - 1;
    const double th = kc * ((side < 2) ? g.tfx : g.tfy);
    double out;
    if (inner) {
      const int nb = (side == 0) ? l - 1 : (side == 1) ? l + 1 : (side == 2) ? l - M : l + M;
      const double tn = kap[nb] * ((side < 2) ? g.tfx : g.tfy);
      const double T = series2(th, tn);
      out = T * dd_diff(pv, 0.0, ph[nb], 0.0);
      if (a.rho && side >= 2) {
        const size_t c = (size_t)j * g.nx + i;
        out += grav_out(g, side, T, 0.5 * g.hy, a.rho[c] + a.rho[side == 2 ? c - g.nx : c + g.nx]);
      }
    } else {
      const int e = side_iface(g, I, J, side);
      if (e >= 0) {
        out = Fout[side][(side < 2) ? lj : li];
      } else {
        const double flen = (side < 2) ? g.hy : g.hx;
        const double v = a.bcv[side][(side < 2) ? j : i];
        out = (g.kind[side] == 1) ? th * dd_diff(pv, 0.0, v, 0.0) : v * flen;
        if (a.rho && g.kind[side] == 1) out += grav_out(g, side, th, 0.5 * g.hy, a.rho[(size_t)j * g.nx + i]);
      }
    }
    dd_add(hi, lo, -out);
  }
  if (l == 0 && tp != 0.0) dd_add(hi, lo, -tp * dd_diff(pv, 0.0, pref, 0.0));
  return hi + lo;
}

// Traces of every column projected on the interface functions: the
// subdomain's block of the interface system, rows of flux dofs negated (the
// form in which the assembled interface matrix is symmetric), last column =
// right-hand side.  Column col of the local solutions at cell l is
// Xs[l * ls + col * cs] (cell-major in LDS or scratch, or the column-major
// output array); all threads of the work-group take part.  win >= 0: only
// the columns of dofs 4 win .. 4 win + 3 of each side (and the right-hand
// side for window 0), the ones that window's work-group solved.
template <int M, int D>
__device__ void generic_block(const SubArgs& a, int sd, int I, int J, const double* kap,
                              const double* Xs, int ls, int cs, int win = -1) {
  constexpr int NBR = 4 * D, NBC = 4 * D + 1;
  const Geo& g = a.g;
  double* blk = a.blocks + (size_t)sd * NBR * NBC;
  const int nP = g.nP;
  int e0side = -1;      // side holding global dof 0 (gauge), if any
  bool e0lo = false;
  if (g.gauge) {
    for (int side = 0; side < 4; ++side)
      if (side_iface(g, I, J, side) == 0) { e0side = side; e0lo = side_sigma(side) > 0; }
  }
  for (int o = threadIdx.x; o < NBR * NBC; o += blockDim.x) {
    const int r = o / NBC, qc = o % NBC;
    if (win >= 0 && (qc < NBR ? ((qc % D) >> 2) != win : win != 0)) continue;
    const int side = r / D, k = r % D;
    const int e = side_iface(g, I, J, side);
    double val = 0.0;
    if (e >= 0) {
      const int col = (qc < NBR) ? 1 + qc : 0;
      const SideGeo sg = side_geo(g, side);
      const double al = a.alpha[e];
      const double sig = side_sigma(side);
      const double* bs = a.basis + (size_t)e * D * M;
      const bool colside = col >= 1 + side * D && col < 1 + side * D + D;
      const int kc = col - 1 - side * D;
      double sum = 0.0;
      for (int t = 0; t < M; ++t) {
        const int l = side_cell<M>(side, t);
        const double kk = kap[l];
        const double TR = sg.flen * kk / (sg.dist + al * sg.H);
        const double beta = al * sg.H / kk;
        double gv = 0.0;
        if (colside) gv = (kc < nP) ? bs[kc * M + t] : -beta * sig * bs[kc * M + t];
        double F = TR * (Xs[(size_t)l * ls + (size_t)col * cs] - gv);
        if (col == 0 && a.rho)
          F += robin_grav(a, side, (size_t)(J * M + l / M) * g.nx + I * M + l % M, TR, sg.dist);
        if (k < nP) sum += bs[k * M + t] * F;
        else sum += bs[k * M + t] * (gv + beta * F / sg.flen);
      }
      const double natural = (k < nP) ? sum : sig * sg.flen * sum;
      const double sgn = (k < nP) ? 1.0 : -1.0;
      val = (qc < NBR) ? sgn * natural : -sgn * natural;
      if (e0side >= 0) {
        const int r0 = e0side * D;   // local position of global dof 0
        if (r == r0) val = (qc == r0 && e0lo) ? 1.0 : 0.0;
        else if (qc == r0) val = 0.0;
      }
      if (a.nact) {
        // slots beyond the interface's functions: their row and column are
        // zero, and the lower-index side puts 1 on the diagonal (the dof
        // is then 0)
        if (!slot_active(a, e, k)) val = (qc == r && side_sigma(side) > 0) ? 1.0 : 0.0;
        else if (qc < NBR) {
          const int es = side_iface(g, I, J, qc / D);
          if (es >= 0 && !slot_active(a, es, qc % D)) val = 0.0;
        }
      }
    }
    blk[o] = val;
  }
}

template <int M>
__device__ void load_kappa(const SubArgs& a, int I, int J, double* kap) {
  const Geo& g = a.g;
  for (int l = threadIdx.x; l < M * M; l += blockDim.x) {
    const int li = l % M, lj = l / M;
    const size_t c = (size_t)(J * M + lj) * g.nx + I * M + li;
    const double lam = a.lam[c];
    if (!(lam > 0.0) || !isfinite(lam)) atomicOr(a.status, ST_BAD_LAMBDA);
    kap[l] = a.K[c] * lam;
  }
}

}  // namespace local
}  // namespace mrcm
