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
// work-group in LDS.  Larger fronts (the few nodes near the root) are
// gathered in global memory and eliminated by a right-looking blocked LU:
// the gather factors the first panel's diagonal block; then one launch per
// panel of PANEL_NB columns applies the trailing update
// A22 -= (A21 U11^-1)(L11^-1 A12) in 64x64 tiles, and the work-group whose
// tile starts with the next panel's diagonal block factors it and stores the
// inverses of its two triangular factors.  Back substitution runs top down,
// one work-group per node.
#include "mrcm_internal.h"

#include <math.h>

namespace mrcm {

namespace {

constexpr int NT = 256;

__device__ inline double gather_entry(const NodeDesc& nd, const double* tree, int2 ma, int2 mb,
                                      bool rhs) {
  double v = 0.0;
  if (!rhs) {
    if (ma.x >= 0 && mb.x >= 0) v += tree[nd.c_off[0] + (long long)ma.x * nd.c_ld[0] + mb.x];
    if (ma.y >= 0 && mb.y >= 0) v += tree[nd.c_off[1] + (long long)ma.y * nd.c_ld[1] + mb.y];
  } else {
    if (ma.x >= 0) v += tree[nd.c_off[0] + (long long)ma.x * nd.c_ld[0] + nd.c_rhs[0]];
    if (ma.y >= 0) v += tree[nd.c_off[1] + (long long)ma.y * nd.c_ld[1] + nd.c_rhs[1]];
  }
  return v;
}

// 2-D thread map used by the element loops below (no integer division):
// 32 columns x 8 rows per pass.
constexpr int TXN = 32, TYN = NT / TXN;

__global__ void __launch_bounds__(NT) front_small_kernel(const NodeDesc* nodes, const int* ids,
                                                         double* tree, const int2* maps,
                                                         int* status) {
  extern __shared__ double F[];
  const NodeDesc nd = nodes[ids[blockIdx.x]];
  const int n = nd.n, s = nd.s, ld = n + 1;
  const int tid = threadIdx.x, tx = tid % TXN, ty = tid / TXN;
  const int2* mp = maps + nd.map_off;
  for (int a = ty; a < n; a += TYN) {
    const int2 ma = mp[a];
    for (int b = tx; b <= n; b += TXN) F[a * ld + b] = gather_entry(nd, tree, ma, b < n ? mp[b] : ma, b == n);
  }
  __syncthreads();
  bool bad = false;
  for (int k = 0; k < s; ++k) {
    const double piv = F[k * ld + k];
    if (piv == 0.0 || !isfinite(piv)) bad = true;
    const double ip = 1.0 / piv;
    for (int a = k + 1 + tid; a < n; a += NT) F[a * ld + k] *= ip;
    __syncthreads();
    for (int a = k + 1 + ty; a < n; a += TYN) {
      const double f = F[a * ld + k];
      for (int b = k + 1 + tx; b <= n; b += TXN) F[a * ld + b] -= f * F[k * ld + b];
    }
    __syncthreads();
  }
  double* out = tree + nd.f_off;
  for (int a = ty; a < n; a += TYN)
    for (int b = tx; b <= n; b += TXN) out[(long long)a * ld + b] = F[a * ld + b];
  if (bad && tid == 0) atomicOr(status, ST_IFACE_PIVOT);
}

// LU without pivoting of the diagonal block of a panel held in LDS
// (identity-padded beyond nb), written back to F at (k0, k0), and the
// explicit inverses of its unit lower factor L11 and upper factor U11,
// stored for the panel in `out` (2 * PANEL_NB^2 doubles).  Every thread of
// the work-group must call it; each inverse column is built in registers by
// one thread.
__device__ void factor_store_diag(double (*A)[PANEL_NB + 1], int nb, double* F, int ld, int k0,
                                  double* out, bool& bad) {
  const int t = threadIdx.x, tx = t % TXN, ty = t / TXN;
  __syncthreads();
  for (int k = 0; k < nb; ++k) {
    const double piv = A[k][k];
    if (piv == 0.0 || !isfinite(piv)) bad = true;
    if (t > k && t < PANEL_NB) A[t][k] /= piv;
    __syncthreads();
    for (int i = k + 1 + ty; i < PANEL_NB; i += TYN)
      if (tx > k) A[i][tx] -= A[i][k] * A[k][tx];
    __syncthreads();
  }
  for (int i = ty; i < nb; i += TYN)
    if (tx < nb) F[(long long)(k0 + i) * ld + k0 + tx] = A[i][tx];
  if (t < PANEL_NB) {
    const int j = t;      // column j of L11^{-1} (unit lower): forward substitution of e_j
    double x[PANEL_NB];
#pragma unroll
    for (int i = 0; i < PANEL_NB; ++i) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int m = 0; m < i; ++m) v -= A[i][m] * x[m];
      x[i] = (i < j) ? 0.0 : v;
    }
#pragma unroll
    for (int i = 0; i < PANEL_NB; ++i) out[i * PANEL_NB + j] = x[i];
  } else if (t >= 64 && t < 64 + PANEL_NB) {
    const int j = t - 64; // column j of U11^{-1} (upper): back substitution of e_j
    double x[PANEL_NB];
#pragma unroll
    for (int i = PANEL_NB - 1; i >= 0; --i) {
      double v = (i == j) ? 1.0 : 0.0;
#pragma unroll
      for (int m = i + 1; m < PANEL_NB; ++m) v -= A[i][m] * x[m];
      x[i] = (i > j) ? 0.0 : v / A[i][i];
    }
#pragma unroll
    for (int i = 0; i < PANEL_NB; ++i) out[PANEL_NB * PANEL_NB + i * PANEL_NB + j] = x[i];
  }
}

__device__ inline double* panel_inv(double* inv, const NodeDesc& nd, int k0) {
  return inv + nd.inv_off + (long long)(k0 / PANEL_NB) * 2 * PANEL_NB * PANEL_NB;
}

// items: (node index, first row); each work-group gathers PANEL_NB rows of
// a blocked front.  The work-group of rows 0 .. PANEL_NB-1 also factors the
// diagonal block of the first panel.
__global__ void __launch_bounds__(NT) front_gather_kernel(const NodeDesc* nodes, const int2* items,
                                                          double* tree, const int2* maps,
                                                          double* inv, int* status) {
  __shared__ double A[PANEL_NB][PANEL_NB + 1];
  const int2 it = items[blockIdx.x];
  const NodeDesc nd = nodes[it.x];
  const int n = nd.n, ld = n + 1;
  const int2* mp = maps + nd.map_off;
  const int r0 = it.y, r1 = min(n, r0 + PANEL_NB);
  const int tx = threadIdx.x % TXN, ty = threadIdx.x / TXN;
  double* F = tree + nd.f_off;
  const bool first = (r0 == 0);
  const int nb = min(PANEL_NB, nd.s);
  for (int a = r0 + ty; a < r0 + PANEL_NB; a += TYN) {
    if (a < r1) {
      const int2 ma = mp[a];
      for (int b = tx; b <= n; b += TXN) {
        const double v = gather_entry(nd, tree, ma, b < n ? mp[b] : ma, b == n);
        F[(long long)a * ld + b] = v;
        if (first && b < PANEL_NB) A[a][b] = (a < nb && b < nb) ? v : (a == b ? 1.0 : 0.0);
      }
    } else if (first) {
      A[a][tx] = (a == tx) ? 1.0 : 0.0;
    }
  }
  if (first) {
    bool bad = false;
    factor_store_diag(A, nb, F, ld, 0, panel_inv(inv, nd, 0), bad);
    if (bad && threadIdx.x == 0) atomicOr(status, ST_IFACE_PIVOT);
  }
}

// Diagonal block of the first panel of blocked fronts (used when a front
// is not gathered by front_gather_kernel).  One work-group per front.
__global__ void __launch_bounds__(NT) front_diag_kernel(const NodeDesc* nodes, const int* ids,
                                                        int k0, double* tree, double* inv,
                                                        int* status) {
  __shared__ double A[PANEL_NB][PANEL_NB + 1];
  const NodeDesc nd = nodes[ids[blockIdx.x]];
  const int ld = nd.n + 1;
  const int nb = min(PANEL_NB, nd.s - k0);
  double* F = tree + nd.f_off;
  const int t = threadIdx.x, tx = t % TXN, ty = t / TXN;
  for (int i = ty; i < PANEL_NB; i += TYN)
    A[i][tx] = (i < nb && tx < nb) ? F[(long long)(k0 + i) * ld + k0 + tx] : (i == tx ? 1.0 : 0.0);
  bool bad = false;
  factor_store_diag(A, nb, F, ld, k0, panel_inv(inv, nd, k0), bad);
  if (bad && t == 0) atomicOr(status, ST_IFACE_PIVOT);
}

// Trailing update of panel k0 for one 64 x 64 tile of a blocked front:
// L21 = A21 U11^{-1} and U12 = L11^{-1} A12 are formed on the fly for the
// tile's rows and columns, then A22 -= L21 U12.  The panel rows and columns
// themselves are left as they were at the start of the panel (back
// substitution applies L11^{-1} and U11^{-1} to them), so tiles never write
// what other tiles read.
__global__ void __launch_bounds__(NT) front_update_kernel(const NodeDesc* nodes,
                                                          const PanelItem* items, int k0,
                                                          double* tree, double* inv,
                                                          int* status) {
  __shared__ double Li[PANEL_NB][PANEL_NB + 1];
  __shared__ double Ui[PANEL_NB][PANEL_NB + 1];
  __shared__ double As[TILE][PANEL_NB + 1];   // A21 tile, then L21
  __shared__ double Bs[PANEL_NB][TILE + 1];   // A12 tile, then U12
  __shared__ double Ls[TILE][PANEL_NB + 1];
  __shared__ double Us[PANEL_NB][TILE + 1];
  const PanelItem it = items[blockIdx.x];
  const NodeDesc nd = nodes[it.node];
  const int n = nd.n, ld = n + 1;
  const int nb = min(PANEL_NB, nd.s - k0);
  double* F = tree + nd.f_off;
  const double* iv = panel_inv(inv, nd, k0);
  const int t = threadIdx.x;
  const int r0 = it.i0, c0 = it.j0;
  const int rows = min(TILE, n - r0), cols = min(TILE, ld - c0);
  for (int e = t; e < PANEL_NB * PANEL_NB; e += NT) {
    Li[e / PANEL_NB][e % PANEL_NB] = iv[e];
    Ui[e / PANEL_NB][e % PANEL_NB] = iv[PANEL_NB * PANEL_NB + e];
  }
  for (int e = t; e < TILE * PANEL_NB; e += NT) {
    const int i = e / PANEL_NB, k = e % PANEL_NB;
    As[i][k] = (i < rows && k < nb) ? F[(long long)(r0 + i) * ld + k0 + k] : 0.0;
  }
  for (int e = t; e < PANEL_NB * TILE; e += NT) {
    const int k = e / TILE, j = e % TILE;
    Bs[k][j] = (k < nb && j < cols) ? F[(long long)(k0 + k) * ld + c0 + j] : 0.0;
  }
  __syncthreads();
  // L21 = A21 Ui (upper), U12 = Li (unit lower) A12
  for (int e = t; e < TILE * PANEL_NB; e += NT) {
    const int i = e / PANEL_NB, k = e % PANEL_NB;
    double v = 0.0;
#pragma unroll 8
    for (int m = 0; m < PANEL_NB; ++m) v += As[i][m] * Ui[m][k];
    Ls[i][k] = v;
  }
  for (int e = t; e < PANEL_NB * TILE; e += NT) {
    const int k = e / TILE, j = e % TILE;
    double v = 0.0;
#pragma unroll 8
    for (int m = 0; m < PANEL_NB; ++m) v += Li[k][m] * Bs[m][j];
    Us[k][j] = v;
  }
  __syncthreads();
  const int tx = t % 16, ty = t / 16;
  double acc[4][4] = {};
#pragma unroll 2
  for (int k = 0; k < PANEL_NB; ++k) {
    double lv[4], uv[4];
    for (int u = 0; u < 4; ++u) lv[u] = Ls[ty * 4 + u][k];
    for (int v = 0; v < 4; ++v) uv[v] = Us[k][tx * 4 + v];
    for (int u = 0; u < 4; ++u)
      for (int v = 0; v < 4; ++v) acc[u][v] += lv[u] * uv[v];
  }
  const bool next_diag = it.pad != 0;   // this tile starts with the next panel's diagonal block
  __syncthreads();
  for (int u = 0; u < 4; ++u) {
    const int i = ty * 4 + u;
    for (int v = 0; v < 4; ++v) {
      const int j = tx * 4 + v;
      double val = 0.0;
      if (i < rows && j < cols) {
        val = F[(long long)(r0 + i) * ld + c0 + j] - acc[u][v];
        F[(long long)(r0 + i) * ld + c0 + j] = val;
      }
      if (next_diag && i < PANEL_NB && j < PANEL_NB) Li[i][j] = val;   // reuse as staging
    }
  }
  if (next_diag) {
    const int k1 = k0 + nb, nb1 = min(PANEL_NB, nd.s - k1);
    __syncthreads();
    for (int e = t; e < PANEL_NB * PANEL_NB; e += NT) {
      const int i = e / PANEL_NB, j = e % PANEL_NB;
      if (!(i < nb1 && j < nb1)) Li[i][j] = (i == j) ? 1.0 : 0.0;
    }
    bool bad = false;
    factor_store_diag(Li, nb1, F, ld, k1, panel_inv(inv, nd, k1), bad);
    if (bad && t == 0) atomicOr(status, ST_IFACE_PIVOT);
  }
}

// Back substitution of one front, top down in the tree: x_s from the
// front's eliminated rows and the x_r of its ancestors.
//  classic fronts: row k holds U (upper part) at elimination time k;
//  blocked fronts: the rows of panel p hold L11\U11 on the diagonal block and
//  the panel-time A12 to the right, so x_1 = U11^{-1} L11^{-1} (b_1 - A12 x_2).
__global__ void __launch_bounds__(NT) front_back_kernel(const NodeDesc* nodes, const int* ids,
                                                        const double* tree, const double* inv,
                                                        const int* dofs, double* x) {
  extern __shared__ double xl[];   // n values: front-local unknowns
  __shared__ double y[PANEL_NB], z[PANEL_NB];
  const NodeDesc nd = nodes[ids[blockIdx.x]];
  const int n = nd.n, s = nd.s, ld = n + 1;
  const double* F = tree + nd.f_off;
  const int* dof = dofs + nd.dof_off;
  const int t = threadIdx.x;
  for (int m = s + t; m < n; m += NT) xl[m] = x[dof[m]];
  __syncthreads();
  if (!nd.blocked) {
    for (int k0 = 0; k0 < s; k0 += NT / 8) {
      const int k = k0 + t / 8, lane = t % 8;
      double v = 0.0;
      if (k < s) {
        const double* row = F + (long long)k * ld;
        for (int m = s + lane; m < n; m += 8) v -= row[m] * xl[m];
        if (lane == 0) v += row[n];
      }
      for (int off = 4; off > 0; off >>= 1) v += __shfl_down(v, off, 8);
      if (k < s && lane == 0) xl[k] = v;
    }
    __syncthreads();
    for (int k = s - 1; k >= 0; --k) {
      const double xk = xl[k] / F[(long long)k * ld + k];
      __syncthreads();
      for (int i = t; i < k; i += NT) xl[i] -= F[(long long)i * ld + k] * xk;
      if (t == 0) xl[k] = xk;
      __syncthreads();
    }
  } else {
    const int np = (s + PANEL_NB - 1) / PANEL_NB;
    for (int p = np - 1; p >= 0; --p) {
      const int k0 = p * PANEL_NB, nb = min(PANEL_NB, s - k0);
      // y = b_1 - A12 x_2: 8 lanes per row, then a reduction across them
      {
        const int row = t / 8, lane = t % 8;
        double v = 0.0;
        if (row < nb) {
          const double* fr = F + (long long)(k0 + row) * ld;
          for (int m = k0 + nb + lane; m < n; m += 8) v -= fr[m] * xl[m];
          if (lane == 0) v += fr[n];
        }
        for (int off = 4; off > 0; off >>= 1) v += __shfl_down(v, off, 8);
        if (row < nb && lane == 0) y[row] = v;
      }
      __syncthreads();
      const double* Li = inv + nd.inv_off + (long long)p * 2 * PANEL_NB * PANEL_NB;
      const double* Ui = Li + PANEL_NB * PANEL_NB;
      if (t < nb) {
        double v = 0.0;
        for (int m = 0; m <= t; ++m) v += Li[t * PANEL_NB + m] * y[m];
        z[t] = v;
      }
      __syncthreads();
      if (t < nb) {
        double v = 0.0;
        for (int m = t; m < nb; ++m) v += Ui[t * PANEL_NB + m] * z[m];
        xl[k0 + t] = v;
      }
      __syncthreads();
    }
  }
  for (int k = t; k < s; k += NT) x[dof[k]] = xl[k];
}

// r = b - A x gathered from the subdomain blocks (each interface row has
// two owners: its lower- and higher-index subdomain).  Stage 1: per
// work-group maxima of |r| and |b|; stage 2: one work-group reduces them.
__global__ void __launch_bounds__(NT) iface_residual_kernel(Geo g, const double* blocks,
                                                            const double* x, double* partials) {
  __shared__ double red[2][NT];
  const int D = g.D, NBR = 4 * D, NBC = NBR + 1;
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
    double ax = 0.0, b = 0.0;
    for (int o = 0; o < 2; ++o) {
      const int sd = sub[o];
      const int I = sd % g.SX, J = sd / g.SX;
      const double* blk = blocks + (size_t)sd * NBR * NBC + (size_t)(side[o] * D + k) * NBC;
      b += blk[NBR];
      for (int sd_side = 0; sd_side < 4; ++sd_side) {
        int ee;
        switch (sd_side) {
          case 0: ee = I > 0 ? J * (g.SX - 1) + I - 1 : -1; break;
          case 1: ee = I < g.SX - 1 ? J * (g.SX - 1) + I : -1; break;
          case 2: ee = J > 0 ? g.nV + (J - 1) * g.SX + I : -1; break;
          default: ee = J < g.SY - 1 ? g.nV + J * g.SX + I : -1;
        }
        if (ee < 0) continue;
        for (int kk = 0; kk < D; ++kk) ax += blk[sd_side * D + kk] * x[(size_t)ee * D + kk];
      }
    }
    rmax = fmax(rmax, fabs(b - ax));
    bmax = fmax(bmax, fabs(b));
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
                                                       double* out2) {
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
  }
}

}  // namespace

hipError_t prepare_interface_kernels() {
  return hipFuncSetAttribute((const void*)front_small_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize,
                             SMALL_FRONT * (SMALL_FRONT + 1) * (int)sizeof(double));
}

hipError_t launch_front_small(const NodeDesc* nodes, const int* ids, int count, int max_n,
                              double* tree, const int2* maps, int* status, hipStream_t st) {
  const size_t lds = (size_t)max_n * (max_n + 1) * sizeof(double);
  hipLaunchKernelGGL(front_small_kernel, dim3(count), dim3(NT), lds, st, nodes, ids, tree, maps,
                     status);
  return hipGetLastError();
}

hipError_t launch_front_gather(const NodeDesc* nodes, const int2* items, int count, double* tree,
                               const int2* maps, double* inv, int* status, hipStream_t st) {
  hipLaunchKernelGGL(front_gather_kernel, dim3(count), dim3(NT), 0, st, nodes, items, tree, maps,
                     inv, status);
  return hipGetLastError();
}

hipError_t launch_front_diag(const NodeDesc* nodes, const int* ids, int count, int k0,
                             double* tree, double* inv, int* status, hipStream_t st) {
  hipLaunchKernelGGL(front_diag_kernel, dim3(count), dim3(NT), 0, st, nodes, ids, k0, tree, inv,
                     status);
  return hipGetLastError();
}

hipError_t launch_front_update(const NodeDesc* nodes, const PanelItem* items, int count, int k0,
                               double* tree, double* inv, int* status, hipStream_t st) {
  hipLaunchKernelGGL(front_update_kernel, dim3(count), dim3(NT), 0, st, nodes, items, k0, tree,
                     inv, status);
  return hipGetLastError();
}

hipError_t launch_front_back(const NodeDesc* nodes, const int* ids, int count, const double* tree,
                             const double* inv, const int* dofs, double* x, hipStream_t st) {
  // callers guarantee n <= 4096 (32 KiB of LDS)
  hipLaunchKernelGGL(front_back_kernel, dim3(count), dim3(NT), 4096 * sizeof(double), st, nodes,
                     ids, tree, inv, dofs, x);
  return hipGetLastError();
}

hipError_t launch_iface_residual(const Geo& g, const double* blocks, const double* x,
                                 double* partials, double* out2, hipStream_t st) {
  hipLaunchKernelGGL(iface_residual_kernel, dim3(RESID_WG), dim3(NT), 0, st, g, blocks, x,
                     partials);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(max_pairs_kernel, dim3(1), dim3(NT), 0, st, partials, RESID_WG, out2);
  return hipGetLastError();
}

}  // namespace mrcm
