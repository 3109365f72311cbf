// Per-subdomain kernels of the MRCM Darcy solve (gfx950).
//
//  * local_basis_kernel: one work-group per subdomain assembles the local
//    Robin problem (paper, section 3, eq. (mrc1) with the Robin parameter of
//    eq. (beta)) from the current mobility, factors it and solves it for the
//    particular solution and one basis function per interface dof (the
//    multiscale basis of section 3), then projects the traces of every
//    column on the interface functions, which gives the subdomain's block of
//    the interface system (eq. (mrc2)).
//  * stitch_kernel: composes the cell pressure from the basis functions and
//    the interface solution, averages the two one-sided Robin fluxes on the
//    skeleton and re-solves each subdomain with that flux as Neumann data
//    (the flux downscaling step the paper cites for continuous interface
//    fluxes), writes the fine fluxes and the per-cell mass balance.
//
// Local matrix: cell-centred two-point scheme in the natural row-major
// ordering of the subdomain, i.e. block tridiagonal with M x M blocks:
// tridiagonal diagonal blocks D_j (couplings along x inside row j) and
// diagonal off-diagonal blocks C_j (couplings along y between rows j and
// j+1).  It is solved by block elimination along the rows with explicit
// inverses of the Schur-complemented diagonal blocks:
//     S_0 = D_0,  S_j = D_j - C_{j-1} S_{j-1}^{-1} C_{j-1},
//     Z_j = S_j^{-1} (B_j - C_{j-1} Z_{j-1}),
//     X_{M-1} = Z_{M-1},  X_j = Z_j - S_j^{-1} C_j X_{j+1}.
// Because C_j is diagonal, the Schur update is an element-wise scaling and
// every other step is a small dense product.  The inverses come from
// Gauss-Jordan sweeps on the symmetric positive definite S_j (no pivoting
// needed); each thread keeps one element of S_j in a register and only the
// pivot row and column go through LDS.
#include "local_common.h"

namespace mrcm {

namespace {

constexpr int NT = 256;
constexpr int LOCAL_IR_STEPS = 3;   // refinement steps of the local basis solve
using namespace local;

// Block elimination of the local system for NR right-hand sides held in
// Xs[MM][NR]; leaves the solution in Xs and the inverse Schur blocks in
// Sinv[M][MM] (LDS, or global scratch for large M).  Each thread keeps
// EPT elements of S_j in registers.  T is the working precision (double,
// or float for the FP32 factorisation of a scaled matrix).  Returns true
// (on every thread) if a pivot was not positive.
template <int M, int NR, class T>
__device__ bool thomas_solve(T* Xs, T* Sinv, const T* dg, const T* ex, const T* cy,
                             T* pivbuf /*[2][2][M]*/) {
  constexpr int MM = M * M;
  constexpr int NQ = (M * NR + NT - 1) / NT;
  constexpr int EPT = (MM + NT - 1) / NT;
  const int tid = threadIdx.x;
  T s[EPT];
  int ta[EPT], tb[EPT];
  bool own[EPT];
#pragma unroll
  for (int q = 0; q < EPT; ++q) {
    const int e = tid + q * NT;
    own[q] = e < MM;
    ta[q] = e / M;
    tb[q] = e % M;
    s[q] = T(0);
  }
  int par = 0;
  bool bad = false;
  T acc[NQ];
  for (int j = 0; j < M; ++j) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      if (!own[q]) continue;
      const int a_ = ta[q], b_ = tb[q];
      T dv = (a_ == b_) ? dg[j * M + a_]
           : (b_ == a_ + 1) ? ex[j * M + a_]
           : (a_ == b_ + 1) ? ex[j * M + b_] : T(0);
      if (j > 0) dv -= cy[(j - 1) * M + a_] * s[q] * cy[(j - 1) * M + b_];
      s[q] = dv;
    }
    for (int k = 0; k < M; ++k) {
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        if (own[q] && tb[q] == k) pivbuf[(par * 2 + 0) * M + ta[q]] = s[q];
        if (own[q] && ta[q] == k) pivbuf[(par * 2 + 1) * M + tb[q]] = s[q];
      }
      __syncthreads();
      const T p = pivbuf[(par * 2 + 1) * M + k];
      if (!(p > T(0))) bad = true;
      const T ip = T(1) / p;
#pragma unroll
      for (int q = 0; q < EPT; ++q) {
        if (!own[q]) continue;
        const T sak = pivbuf[(par * 2 + 0) * M + ta[q]];
        const T skb = pivbuf[(par * 2 + 1) * M + tb[q]];
        if (ta[q] == k && tb[q] == k) s[q] = ip;
        else if (ta[q] == k) s[q] = s[q] * ip;
        else if (tb[q] == k) s[q] = -sak * ip;
        else s[q] = s[q] - sak * skb * ip;
      }
      par ^= 1;
    }
#pragma unroll
    for (int q = 0; q < EPT; ++q)
      if (own[q]) Sinv[j * MM + tid + q * NT] = s[q];
    __syncthreads();
    // Z_j = S_j^{-1} (B_j - C_{j-1} Z_{j-1})
    {
      int q = 0;
      for (int o = tid; o < M * NR; o += NT, ++q) {
        const int ra = o / NR, col = o % NR;
        T sum = T(0);
        for (int b = 0; b < M; ++b) {
          T r = Xs[(j * M + b) * NR + col];
          if (j > 0) r -= cy[(j - 1) * M + b] * Xs[((j - 1) * M + b) * NR + col];
          sum += Sinv[j * MM + ra * M + b] * r;
        }
        acc[q] = sum;
      }
      __syncthreads();
      q = 0;
      for (int o = tid; o < M * NR; o += NT, ++q) {
        const int ra = o / NR, col = o % NR;
        Xs[(j * M + ra) * NR + col] = acc[q];
      }
    }
  }
  __syncthreads();
  for (int j = M - 2; j >= 0; --j) {
    int q = 0;
    for (int o = tid; o < M * NR; o += NT, ++q) {
      const int ra = o / NR, col = o % NR;
      T sum = Xs[(j * M + ra) * NR + col];
      for (int b = 0; b < M; ++b)
        sum -= Sinv[j * MM + ra * M + b] * cy[j * M + b] * Xs[((j + 1) * M + b) * NR + col];
      acc[q] = sum;
    }
    q = 0;
    for (int o = tid; o < M * NR; o += NT, ++q) {
      const int ra = o / NR, col = o % NR;
      Xs[(j * M + ra) * NR + col] = acc[q];
    }
    __syncthreads();
  }
  return bad;
}

// Solve again with the inverse Schur blocks already in Sinv (no factoring):
// the forward and backward block sweeps of thomas_solve on NR new columns.
template <int M, int NR, class T>
__device__ void thomas_resolve(T* Xs, const T* Sinv, const T* cy) {
  constexpr int MM = M * M;
  constexpr int NQ = (M * NR + NT - 1) / NT;
  const int tid = threadIdx.x;
  T acc[NQ];
  __syncthreads();
  for (int j = 0; j < M; ++j) {
    int q = 0;
    for (int o = tid; o < M * NR; o += NT, ++q) {
      const int ra = o / NR, col = o % NR;
      T sum = T(0);
      for (int b = 0; b < M; ++b) {
        T r = Xs[(j * M + b) * NR + col];
        if (j > 0) r -= cy[(j - 1) * M + b] * Xs[((j - 1) * M + b) * NR + col];
        sum += Sinv[j * MM + ra * M + b] * r;
      }
      acc[q] = sum;
    }
    __syncthreads();
    q = 0;
    for (int o = tid; o < M * NR; o += NT, ++q) {
      const int ra = o / NR, col = o % NR;
      Xs[(j * M + ra) * NR + col] = acc[q];
    }
    __syncthreads();
  }
  for (int j = M - 2; j >= 0; --j) {
    int q = 0;
    for (int o = tid; o < M * NR; o += NT, ++q) {
      const int ra = o / NR, col = o % NR;
      T sum = Xs[(j * M + ra) * NR + col];
      for (int b = 0; b < M; ++b)
        sum -= Sinv[j * MM + ra * M + b] * cy[j * M + b] * Xs[((j + 1) * M + b) * NR + col];
      acc[q] = sum;
    }
    q = 0;
    for (int o = tid; o < M * NR; o += NT, ++q) {
      const int ra = o / NR, col = o % NR;
      Xs[(j * M + ra) * NR + col] = acc[q];
    }
    __syncthreads();
  }
}

// r <- b - A x in double-double for the local five-point matrix, NR columns
// (r may be b); dgl: the rounding error of the diagonal sums, so that the
// residual is the cells' mass balance (flux form) to double-double accuracy
template <int M, int NR>
__device__ void local_residual_dd(const double* b, const double* x, double* r, const double* dg,
                                  const float* dgl, const double* ex, const double* cy) {
  for (int o = threadIdx.x; o < M * M * NR; o += NT) {
    const int l = o / NR, col = o % NR;
    const int li = l % M, lj = l / M;
    double hi = b[o], lo = 0.0;
    dd_fma(hi, lo, -dg[l], x[o]);
    dd_fma_low(lo, -(double)dgl[l], x[o]);
    if (li < M - 1) dd_fma(hi, lo, -ex[l], x[(l + 1) * NR + col]);
    if (li > 0) dd_fma(hi, lo, -ex[l - 1], x[(l - 1) * NR + col]);
    if (lj < M - 1) dd_fma(hi, lo, -cy[l], x[(l + M) * NR + col]);
    if (lj > 0) dd_fma(hi, lo, -cy[l - M], x[(l - M) * NR + col]);
    r[o] = hi + lo;
  }
}

// LDS holds the basis-function block and the inverse Schur blocks up to
// 16 x 16 subdomains; larger ones keep them in the per-subdomain scratch
template <int M>
struct LocalStore {
  static constexpr bool big = M > 16;
  // the inverse Schur blocks in the scratch too: large subdomains, and 16 x 16
  // ones whose basis block (R columns) leaves no LDS for them at two
  // work-groups per CU
  static constexpr bool sinv_global(int R) { return big || M * M * R * 8 > 48 * 1024; }
};

// FP64 local solves (LIST: only the subdomains on the fallback list of the
// FP32 kernel below)
template <int M, int D, bool LIST>
__global__ void __launch_bounds__(NT) local_basis_kernel(SubArgs a) {
  constexpr int R = 1 + 4 * D;
  constexpr int MM = M * M;
  constexpr bool BIG = LocalStore<M>::big;
  // with many columns (8 dofs per interface) the inverse blocks go to the
  // scratch as well, so that two work-groups share a CU
  constexpr bool SG = LocalStore<M>::sinv_global(R);
  __shared__ double kap[MM], dg[MM], ex[MM], cy[MM];
  __shared__ float dgl[MM];            // rounding error of the diagonal sums
  __shared__ double Xs_l[BIG ? 1 : MM * R];
  __shared__ double Sinv_l[SG ? 1 : M * MM];
  __shared__ double pivbuf[4 * M];
  const Geo& g = a.g;
  const int tid = threadIdx.x;
  int sd = blockIdx.x;
  if (LIST) {
    if ((int)blockIdx.x >= a.fallback[0]) return;
    sd = a.fallback[1 + blockIdx.x];
  }
  const int I = sd % g.SX, J = sd / g.SX;
  // per-subdomain scratch: [Bs | Rs] (all sizes), then [Xs | Sinv] beyond
  // 16 x 16; its length is local_scratch_doubles()
  double* scr = a.scratch + (size_t)sd * a.scratch_stride;
  double* Rs_l = scr + MM * R;
  double* Bs = scr;
  double* Xs = BIG ? scr + 2 * MM * R : Xs_l;
  double* Sinv = BIG ? scr + 3 * MM * R : SG ? scr + 2 * MM * R : Sinv_l;

  load_kappa<M>(a, I, J, kap);
  __syncthreads();
  for (int l = tid; l < MM; l += NT)
    assemble_cell<M, R>(a, I, J, l, kap, dg, ex, cy, Xs + l * R, 1, nullptr, dgl);
  __syncthreads();
  for (int o = tid; o < MM * R; o += NT) Bs[o] = Xs[o];

  if (thomas_solve<M, R, double>(Xs, Sinv, dg, ex, cy, pivbuf) && tid == 0)
    atomicOr(a.status, ST_LOCAL_PIVOT);
  // iterative refinement, residual in double-double with the exact diagonal
  // (Bs keeps B; the correction goes through Rg)
  double* Rg = Rs_l;
  for (int it = 0; it < LOCAL_IR_STEPS; ++it) {
    __syncthreads();
    local_residual_dd<M, R>(Bs, Xs, Rg, dg, dgl, ex, cy);
    thomas_resolve<M, R, double>(Rg, Sinv, cy);
    for (int o = tid; o < MM * R; o += NT) Xs[o] += Rg[o];
  }
  __syncthreads();

  double* Xg = a.X + (size_t)sd * MM * R;   // column-major per subdomain: [col][cell]
  for (int o = tid; o < MM * R; o += NT) Xg[(o % R) * MM + o / R] = Xs[o];
  generic_block<M, D>(a, sd, I, J, kap, Xs, R, 1);
}

// FP32 factorisation + double-double-residual refinement for the generic sizes with
// their work arrays in the per-subdomain scratch (32 x 32 subdomains): the
// same method as the 16 x 16 FP32 kernel.  The local matrix is scaled
// symmetrically (Ds A Ds, Ds = diag(A)^-1/2, unit diagonal); the inverse
// Schur blocks and the solves of the scaled system are FP32, the solution
// FP64 and the residuals double-double with the exact diagonal (the cells'
// mass balances).  Refinement stops when the largest correction is below
// a.ir_tol of the largest solution value (at most a.ir_max steps); a
// subdomain that ends above it, or met a bad FP32 pivot, is listed for the
// FP64 re-solve.

template <int M, int D>
__global__ void __launch_bounds__(NT) local_basis32_kernel(SubArgs a) {
  constexpr int R = 1 + 4 * D;
  constexpr int MM = M * M;
  static_assert(LocalStore<M>::big && R <= M, "scratch layout of the large subdomains");
  __shared__ double kap[MM], dg[MM], ex[MM], cy[MM], dsc[MM];
  __shared__ float dgl[MM];            // rounding error of the diagonal sums
  __shared__ float dgs[MM], exs[MM], cys[MM];
  __shared__ float pivbuf[4 * M];
  __shared__ double red[2][NT / 64];
  const Geo& g = a.g;
  const int tid = threadIdx.x;
  const int sd = blockIdx.x;
  const int I = sd % g.SX, J = sd / g.SX;
  // scratch: Bs | Rg | Xs (FP64, MM R each), then FP32 Sinv (M MM) and the
  // FP32 work columns Ws (MM R) in the space of the FP64 inverse blocks
  double* scr = a.scratch + (size_t)sd * a.scratch_stride;
  double* Bs = scr;
  double* Rg = scr + MM * R;
  double* Xs = scr + 2 * MM * R;
  float* Sinv = reinterpret_cast<float*>(scr + 3 * MM * R);
  float* Ws = Sinv + M * MM;

  load_kappa<M>(a, I, J, kap);
  __syncthreads();
  for (int l = tid; l < MM; l += NT)
    assemble_cell<M, R>(a, I, J, l, kap, dg, ex, cy, Bs + l * R, 1, nullptr, dgl);
  __syncthreads();
  for (int l = tid; l < MM; l += NT) dsc[l] = 1.0 / sqrt(dg[l]);
  __syncthreads();
  for (int l = tid; l < MM; l += NT) {
    const int li = l % M, lj = l / M;
    dgs[l] = 1.0f;
    exs[l] = li < M - 1 ? (float)(ex[l] * dsc[l] * dsc[l + 1]) : 0.0f;
    cys[l] = lj < M - 1 ? (float)(cy[l] * dsc[l] * dsc[l + M]) : 0.0f;
  }
  for (int o = tid; o < MM * R; o += NT) Ws[o] = (float)(dsc[o / R] * Bs[o]);
  __syncthreads();
  const bool bad = thomas_solve<M, R, float>(Ws, Sinv, dgs, exs, cys, pivbuf);
  __syncthreads();
  for (int o = tid; o < MM * R; o += NT) Xs[o] = dsc[o / R] * (double)Ws[o];

  int used = 0;
  double rel = 1.0;
  for (int it = 0; it < a.ir_max; ++it) {
    __syncthreads();
    local_residual_dd<M, R>(Bs, Xs, Rg, dg, dgl, ex, cy);
    __syncthreads();
    for (int o = tid; o < MM * R; o += NT) Ws[o] = (float)(dsc[o / R] * Rg[o]);
    thomas_resolve<M, R, float>(Ws, Sinv, cys);
    double cmax = 0.0, xmax = 0.0;
    for (int o = tid; o < MM * R; o += NT) {
      const double dx = dsc[o / R] * (double)Ws[o];
      const double x = Xs[o] + dx;
      Xs[o] = x;
      cmax = fmax(cmax, fabs(dx));
      xmax = fmax(xmax, fabs(x));
    }
    for (int off = 32; off > 0; off >>= 1) {
      cmax = fmax(cmax, __shfl_xor(cmax, off));
      xmax = fmax(xmax, __shfl_xor(xmax, off));
    }
    if ((tid & 63) == 0) {
      red[0][tid >> 6] = cmax;
      red[1][tid >> 6] = xmax;
    }
    __syncthreads();
    cmax = 0.0;
    xmax = 0.0;
    for (int w = 0; w < NT / 64; ++w) {
      cmax = fmax(cmax, red[0][w]);
      xmax = fmax(xmax, red[1][w]);
    }
    used = it + 1;
    rel = cmax / fmax(xmax, 1e-300);
    if (rel <= a.ir_tol) break;
  }
  if (tid == 0) {
    atomicMax(a.ir_iters, used);
    if (bad || !(rel <= a.ir_tol)) {
      const int q = atomicAdd(a.fallback, 1);
      a.fallback[1 + q] = sd;
    }
  }
  __syncthreads();

  double* Xg = a.X + (size_t)sd * MM * R;   // column-major per subdomain: [col][cell]
  for (int o = tid; o < MM * R; o += NT) Xg[(o % R) * MM + o / R] = Xs[o];
  generic_block<M, D>(a, sd, I, J, kap, Xs, R, 1);
}

// ---------------------------------------------------------------------------
// stitch re-solve, composition and fine fluxes
// ---------------------------------------------------------------------------

template <int M, int D>
__device__ double compose_at(const SubArgs& a, int sd, int l) {
  // p at local cell l of subdomain sd = X[sd][l] . [1; coefficients]
  constexpr int R = 1 + 4 * D;
  const Geo& g = a.g;
  const int I = sd % g.SX, J = sd / g.SX;
  const double* xr = a.X + (size_t)sd * M * M * R + l;   // [col][cell]
  double p = xr[0];
  for (int side = 0; side < 4; ++side) {
    const int e = side_iface(g, I, J, side);
    if (e < 0) continue;
    for (int k = 0; k < D; ++k) p += xr[(size_t)(1 + side * D + k) * M * M] * a.coef[(size_t)e * D + k];
  }
  return p;
}

template <int M, int D>
__global__ void __launch_bounds__(NT) stitch_kernel(SubArgs a) {
  if (blockIdx.x == 0 && threadIdx.x == 0) stamp_now(a.stamps + STAMP_FLUX);
  constexpr int MM = M * M;
  __shared__ double kap[MM], dg[MM], ex[MM], cy[MM];
  __shared__ double pm[MM];          // composed multiscale pressure
  __shared__ double Xs[MM];          // stitch right-hand side / pressure
  __shared__ double Rs[MM];          // residual / correction
  __shared__ double Sinv_l[LocalStore<M>::big ? 1 : M * MM];
  __shared__ double pivbuf[4 * M];
  __shared__ double Fout[4][M];      // outflow of this subdomain on its skeleton faces
  __shared__ double red[3][NT];
  const Geo& g = a.g;
  const int tid = threadIdx.x;
  const int sd = blockIdx.x;
  double* Sinv = LocalStore<M>::big ? a.scratch + (size_t)sd * a.scratch_stride : Sinv_l;
  const int I = sd % g.SX, J = sd / g.SX;
  const int nP = g.nP;

  load_kappa<M>(a, I, J, kap);
  for (int l = tid; l < MM; l += NT) pm[l] = compose_at<M, D>(a, sd, l);
  __syncthreads();

  // one-sided Robin fluxes on both sides of every skeleton face of this
  // subdomain, and their average
  for (int o = tid; o < 4 * M; o += NT) {
    const int side = o / M, t = o % M;
    const int e = side_iface(g, I, J, side);
    double fo = 0.0;
    if (e >= 0) {
      const SideGeo sg = side_geo(g, side);
      const double al = a.alpha[e];
      const double* bs = a.basis + (size_t)e * D * M;
      const double* ce = a.coef + (size_t)e * D;
      double PH = 0.0, UH = 0.0;
      for (int k = 0; k < nP; ++k) PH += ce[k] * bs[k * M + t];
      for (int k = nP; k < D; ++k) UH += ce[k] * bs[k * M + t];
      const int l = side_cell<M>(side, t);
      const double sig = side_sigma(side);
      const double ko = kap[l];
      const double TRo = sg.flen * ko / (sg.dist + al * sg.H);
      const double Fown = TRo * (pm[l] - (PH - al * sg.H / ko * sig * UH)) +
                          robin_grav(a, side, (size_t)(J * M + l / M) * g.nx + I * M + l % M, TRo, sg.dist);
      // neighbour across the face
      const int nside = side ^ 1;
      const int nsd = (side == 0) ? sd - 1 : (side == 1) ? sd + 1 : (side == 2) ? sd - g.SX : sd + g.SX;
      const int nI = nsd % g.SX, nJ = nsd / g.SX;
      const int nl = side_cell<M>(nside, t);
      const size_t nc = (size_t)(nJ * M + nl / M) * g.nx + nI * M + nl % M;
      const double kn = a.K[nc] * a.lam[nc];
      const double pn = compose_at<M, D>(a, nsd, nl);
      const double TRn = sg.flen * kn / (sg.dist + al * sg.H);
      const double Fnb = TRn * (pn - (PH - al * sg.H / kn * (-sig) * UH)) + robin_grav(a, nside, nc, TRn, sg.dist);
      fo = 0.5 * (Fown - Fnb);
    }
    Fout[side][t] = fo;
  }
  __syncthreads();
  for (int l = tid; l < MM; l += NT)
    assemble_cell<M, 1>(a, I, J, l, kap, dg, ex, cy, Xs + l, 0, Fout);
  __syncthreads();
  // A subdomain with no Dirichlet face has a Neumann problem, solvable only
  // if its data sum to zero.  The averaged skeleton fluxes meet this to the
  // rounding of the composed solution; that defect (summed in double-double)
  // is removed evenly from the cells' data instead of being left to the
  // pinned cell, and the constant is fixed at cell 0 to the composed
  // multiscale pressure (its pin then carries no flux).
  const bool dir = (I == 0 && g.kind[0] == 1) || (I == g.SX - 1 && g.kind[1] == 1) ||
                   (J == 0 && g.kind[2] == 1) || (J == g.SY - 1 && g.kind[3] == 1);
  double dfc = 0.0, tp = 0.0;
  if (!dir) {   // uniform over the work-group
    double sh = 0.0, sl = 0.0;
    for (int l = tid; l < MM; l += NT) dd_add(sh, sl, Xs[l]);
    red[0][tid] = sh;
    red[1][tid] = sl;
    __syncthreads();
    for (int w = NT / 2; w > 0; w >>= 1) {
      if (tid < w) {
        double h = red[0][tid], lo = red[1][tid];
        dd_add(h, lo, red[0][tid + w]);
        red[0][tid] = h;
        red[1][tid] = lo + red[1][tid + w];
      }
      __syncthreads();
    }
    dfc = (red[0][0] + red[1][0]) / MM;
    tp = dg[0];
    __syncthreads();   // every thread has read the sums and dg[0]
    for (int l = tid; l < MM; l += NT) Xs[l] -= dfc;
    __syncthreads();
    if (tid == 0) {
      dg[0] += tp;
      Xs[0] += tp * pm[0];
    }
  }
  __syncthreads();
  if (thomas_solve<M, 1, double>(Xs, Sinv, dg, ex, cy, pivbuf) && threadIdx.x == 0)
    atomicOr(a.status, ST_STITCH_PIVOT);
  // one step of iterative refinement with the stored inverse blocks; the
  // residual is the cells' mass balance in double-double (the FP64 diagonal
  // sums of the assembled matrix would leave eps * T |p| per cell), and the
  // pressure is kept as the unevaluated sum Xs + Rs (solution + correction)
  // from which the fluxes are formed: the cell balances then hold to the
  // rounding of the fluxes themselves
  __syncthreads();
  for (int l = tid; l < MM; l += NT)
    Rs[l] = stitch_balance_residual<M>(a, I, J, l, kap, Xs, Fout, dfc, tp, pm[0]);
  __syncthreads();
  thomas_resolve<M, 1, double>(Rs, Sinv, cy);
  __syncthreads();

  // fine fluxes (+x / +y) from the stitched pressure; skeleton faces carry
  // the averaged flux.  Each subdomain writes the W and S faces of its cells
  // (and the E / N boundary faces of the last column / row).
  double imb = 0.0, fmx = 0.0, psum = 0.0;
  for (int l = tid; l < MM; l += NT) {
    const int li = l % M, lj = l / M;
    const int i = I * M + li, j = J * M + lj;
    double out[4];
    stitch_out_fluxes<M>(a, I, J, l, kap, Xs, Rs, Fout, out);
    double F[4];  // W, E, S, N in +x / +y direction
    for (int side = 0; side < 4; ++side) F[side] = (side == 0 || side == 2) ? -out[side] : out[side];
    a.ux[(size_t)j * (g.nx + 1) + i] = F[0] / g.hy;
    if (li == M - 1 && I == g.SX - 1) a.ux[(size_t)j * (g.nx + 1) + i + 1] = F[1] / g.hy;
    a.uy[(size_t)j * g.nx + i] = F[2] / g.hx;
    if (lj == M - 1 && J == g.SY - 1) a.uy[(size_t)(j + 1) * g.nx + i] = F[3] / g.hx;
    double q = a.src ? a.src[(size_t)j * g.nx + i] * g.hx * g.hy : 0.0;
    const double net = F[1] - F[0] + F[3] - F[2];
    imb = fmax(imb, fabs(net - q));
    fmx = fmax(fmx, fmax(fmax(fabs(F[0]), fabs(F[1])), fmax(fabs(F[2]), fabs(F[3]))));
    a.p_out[(size_t)j * g.nx + i] = pm[l];
    psum += pm[l];
  }
  red[0][tid] = imb;
  red[1][tid] = fmx;
  red[2][tid] = psum;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] = fmax(red[0][tid], red[0][tid + w]);
      red[1][tid] = fmax(red[1][tid], red[1][tid + w]);
      red[2][tid] = red[2][tid] + red[2][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    a.sub_stats[3 * sd + 0] = red[0][0];
    a.sub_stats[3 * sd + 1] = red[1][0];
    a.sub_stats[3 * sd + 2] = red[2][0];
  }
}

// max imbalance, max |F| and the pressure mean over subdomains (fixed order,
// so the result does not depend on scheduling), then the zero-mean shift of
// the pressure when the problem has no Dirichlet side.
__global__ void __launch_bounds__(NT) finish_reduce_kernel(SubArgs a, double* result) {
  __shared__ double red[3][NT];
  const int tid = threadIdx.x;
  double imb = 0.0, fmx = 0.0, ps = 0.0;
  // CH subdomains per thread loaded before any is used (clamped, dropped
  // beyond the end), summed in the order of s
  constexpr int CH = 16;
  const int ns = a.g.n_sub;
  for (int s0 = tid; s0 < ns; s0 += CH * NT) {
    double v[CH][3];
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      const int s = min(s0 + q * NT, ns - 1);
#pragma unroll
      for (int k = 0; k < 3; ++k) v[q][k] = a.sub_stats[3 * s + k];
    }
#pragma unroll
    for (int q = 0; q < CH; ++q) {
      if (s0 + q * NT < ns) {
        imb = fmax(imb, v[q][0]);
        fmx = fmax(fmx, v[q][1]);
        ps += v[q][2];
      }
    }
  }
  red[0][tid] = imb; red[1][tid] = fmx; red[2][tid] = ps;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (tid < w) {
      red[0][tid] = fmax(red[0][tid], red[0][tid + w]);
      red[1][tid] = fmax(red[1][tid], red[1][tid + w]);
      red[2][tid] += red[2][tid + w];
    }
    __syncthreads();
  }
  if (tid == 0) {
    result[0] = red[0][0] / fmax(red[1][0], 1e-300);
    result[1] = red[2][0] / ((double)a.g.nx * a.g.ny);
    stamp_now(a.stamps + STAMP_FLUX_END);
  }
}

__global__ void shift_kernel(double* p, size_t n, const double* mean) {
  const double m = *mean;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] -= m;
}

__global__ void mobility_kernel(const double* in, double* lam, size_t n, int from_s, double mw,
                                double mo) {
  // four grid strides per step, loaded before any is stored
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i0 = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i0 < n; i0 += 4 * stride) {
    double v[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) v[q] = in[min(i0 + q * stride, n - 1)];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const size_t i = i0 + q * stride;
      if (i < n) lam[i] = from_s ? v[q] * v[q] / mw + (1.0 - v[q]) * (1.0 - v[q]) / mo : v[q];
    }
  }
}

// total mobility and rho = lambda_g / lambda (eq. (fluxos1_wg)) from a
// saturation, for the gravity variant
__global__ void mobility_gravity_kernel(const double* s_in, double* lam, double* rho, size_t n, double mw,
                                        double mo, double rw, double ro) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += stride) {
    const double s = s_in[i];
    const double lw = s * s / mw, lo = (1.0 - s) * (1.0 - s) / mo;
    lam[i] = lw + lo;
    rho[i] = (lw * rw + lo * ro) / (lw + lo);
  }
}

template <int M, int D>
hipError_t launch_pair(const SubArgs& a, hipStream_t st, bool stitch) {
  if (stitch)
    hipLaunchKernelGGL((stitch_kernel<M, D>), dim3(a.g.n_sub), dim3(NT), 0, st, a);
  else
    hipLaunchKernelGGL((local_basis_kernel<M, D, false>), dim3(a.g.n_sub), dim3(NT), 0, st, a);
  return hipGetLastError();
}

// FP32 + refinement, then the FP64 re-solve of the listed subdomains
template <int M, int D>
hipError_t launch_fp32(const SubArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((local_basis32_kernel<M, D>), dim3(a.g.n_sub), dim3(NT), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((local_basis_kernel<M, D, true>), dim3(a.g.n_sub), dim3(NT), 0, st, a);
  return hipGetLastError();
}

hipError_t dispatch(const SubArgs& a, hipStream_t st, bool stitch) {
  const int M = a.g.M, D = a.g.D;
  if (M == 16 && D == 4 && a.g.nP == 2 && !a.g.generic) {
    if (stitch) return launch_stitch_m16d4(a, st);
    if (a.g.prec == 1) {
      hipError_t e = launch_basis32_m16d4(a, st);
      if (e != hipSuccess) return e;
      return launch_basis_m16d4_list(a, st);   // FP64 re-solve of the listed subdomains
    }
    return launch_basis_m16d4(a, st);
  }
  if (M == 16 && D == 8 && !a.g.generic && a.g.prec == 0) {
    return stitch ? launch_stitch_m16d8(a, st) : launch_basis_m16d8(a, st);
  }
  if (M == 32 && D == 8 && basis32x32_supported(a.g))
    return stitch ? launch_stitch32x32(a, st) : launch_basis32x32(a, st, false);
  if (M == 32 && D == 4) {
    if (stitch && basis32x32_supported(a.g)) return launch_stitch32x32(a, st);
    if (!stitch && basis32x32_supported(a.g)) {
      if (a.g.prec == 1) {   // FP32 + refinement, then the FP64 re-solve of the listed ones
        hipLaunchKernelGGL((local_basis32_kernel<32, 4>), dim3(a.g.n_sub), dim3(NT), 0, st, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        return launch_basis32x32(a, st, true);
      }
      return launch_basis32x32(a, st, false);
    }
    if (!stitch && a.g.prec == 1) return launch_fp32<32, 4>(a, st);
    return launch_pair<32, 4>(a, st, stitch);
  }
  if (M == 16 && D == 4) return launch_pair<16, 4>(a, st, stitch);
  if (M == 8 && D == 4) return launch_pair<8, 4>(a, st, stitch);
  if (M == 4 && D == 4) return launch_pair<4, 4>(a, st, stitch);
  if (M == 16 && D == 8) return launch_pair<16, 8>(a, st, stitch);
  if (M == 8 && D == 8) return launch_pair<8, 8>(a, st, stitch);
  if (M == 32 && D == 8) return launch_pair<32, 8>(a, st, stitch);
  if (M == 8 && D == 16) return launch_pair<8, 16>(a, st, stitch);
  if (M == 4 && D == 8) return launch_pair<4, 8>(a, st, stitch);
  return hipErrorInvalidValue;
}

}  // namespace

bool local_fp32_supported(int M, int D, int nP) {
  return (M == 16 && D == 4 && nP == 2) || (M == 32 && D == 4);
}

bool local_supported(int M, int D) {
  return (M == 32 && D == 4) || (M == 16 && D == 4) || (M == 8 && D == 4) || (M == 4 && D == 4) || (M == 8 && D == 16) ||
         (M == 4 && D == 8) || (M == 8 && D == 8) || (M == 16 && D == 8) || (M == 32 && D == 8);
}

long long local_scratch_doubles(const Geo& g) {
  const bool fast = g.M == 16 && ((g.D == 4 && g.nP == 2) || (g.D == 8 && g.prec == 0)) && !g.generic;
  if (fast) return 0;
  // the matrix-core kernels of 32 x 32 subdomains; the FP32 form runs the
  // generic FP32 kernel first and needs its scratch
  if (basis32x32_supported(g) && g.prec != 1) return basis32x32_scratch(g);
  const long long MM = (long long)g.M * g.M, R = 1 + 4 * g.D;
  if (g.M > 16) return 3 * MM * R + g.M * MM;
  return 2 * MM * R + (MM * R * 8 > 48 * 1024 ? g.M * MM : 0);
}

hipError_t launch_local_basis(const SubArgs& a, hipStream_t st) { return dispatch(a, st, false); }

hipError_t launch_stitch(const SubArgs& a, hipStream_t st) { return dispatch(a, st, true); }

hipError_t launch_finish_flux(const SubArgs& a, double* result, hipStream_t st) {
  hipLaunchKernelGGL(finish_reduce_kernel, dim3(1), dim3(NT), 0, st, a, result);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !a.g.gauge) return e;
  const size_t n = (size_t)a.g.nx * a.g.ny;
  hipLaunchKernelGGL(shift_kernel, dim3(1024), dim3(256), 0, st, a.p_out, n, result + 1);
  return hipGetLastError();
}

hipError_t launch_mobility_gravity(const double* s, double* lam, double* rho, size_t n, double mu_w,
                                   double mu_o, double rho_w, double rho_o, hipStream_t st) {
  hipLaunchKernelGGL(mobility_gravity_kernel, dim3(1024), dim3(256), 0, st, s, lam, rho, n, mu_w, mu_o,
                     rho_w, rho_o);
  return hipGetLastError();
}

hipError_t launch_mobility(const double* in, double* lam, size_t n, int from_saturation,
                           double mu_w, double mu_o, hipStream_t st) {
  hipLaunchKernelGGL(mobility_kernel, dim3(1024), dim3(256), 0, st, in, lam, n, from_saturation,
                     mu_w, mu_o);
  return hipGetLastError();
}

}  // namespace mrcm
