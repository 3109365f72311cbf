// Implicit transport of the water saturation (paper, section 4) on the GPU:
// implicit Euler with first-order upwind fluxes (eqs. (BL2D_Newton2),
// (fluxes_impli), (up_fluxes_impli)), Newton's method (eqs. (BL2D_Newton8),
// (BL2D_Newton7)) with the inflection-point strategy, 4 cells per thread.
//
// Per Newton iteration:
//  * assemble_kernel: the residual H and the Jacobian H' of every cell.  A
//    face's water flux depends on the saturation of its upwind cell only, so
//    a cell's row couples it to the neighbours its water comes from.  Rows
//    are scaled by their diagonal (Jacobi), which leaves a unit diagonal,
//    up to four coupling coefficients and the right-hand side -H / diag.
//    A face carries at most one nonzero coupling (in its downstream cell's
//    row), so the couplings are stored one per face.
//  * BiCGSTAB on the scaled system, two fused kernels per iteration (B: s
//    and t = A s; AC: x and r, then the next p and v = A p), each forming
//    the neighbours' values it needs from the previous vectors instead of a
//    separate pass.  The textbook's third reduction, (r^, r) after the r
//    update, is replaced by (r^, s) - omega (r^, t), which kernel B reduces
//    with (t, s) and (t, t).  Inner products are reduced per work-group into
//    partial sums that the next kernel's work-groups all sum in the same
//    fixed order (deterministic, no atomics), so every work-group forms the
//    iteration's scalars itself.  Convergence or breakdown sets a flag in
//    device memory that makes the remaining launches of a batch return at
//    once.
//  * update_kernel (queued after every batch of BiCGSTAB launches, a no-op
//    until the solve has stopped): s <- clamp(s + d) to [0, 1], then the
//    inflection-point rule (an update whose ends lie on different sides of
//    the inflection point of f is halved), and the partial sums of the
//    change's squared L2 norm.
//
// Layout: cell (i, j) at j*nx + i; face velocities as the Darcy step
// returns them (ux on (nx+1)*ny x-faces, uy on nx*(ny+1) y-faces).
#include "transport.h"

#include <math.h>

namespace mrcm {
namespace {

constexpr int TB = 256;   // threads per work-group
constexpr int CPT = 4;    // cells per thread

__device__ inline double fw(double s, double M) {
  const double a = M * s * s, b = (1.0 - s) * (1.0 - s);
  return a / (a + b);
}
__device__ inline double fw_d1(double s, double M) {
  const double d = M * s * s + (1.0 - s) * (1.0 - s);
  return 2.0 * M * s * (1.0 - s) / (d * d);
}
// sign of f'': f' = N / D^2, f'' = (N' D - 2 N D') / D^3 with D > 0
__device__ inline int fw_d2_sign(double s, double M) {
  const double n = 2.0 * M * s * (1.0 - s), dn = 2.0 * M * (1.0 - 2.0 * s);
  const double d = M * s * s + (1.0 - s) * (1.0 - s), dd = 2.0 * M * s - 2.0 * (1.0 - s);
  const double g = dn * d - 2.0 * n * dd;
  return (g > 0.0) - (g < 0.0);
}

// sum over the work-group: wavefront butterflies, then the waves in order
__device__ inline double block_sum(double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < TB / 64; ++k) s += red[k];
  return s;
}

// NV sums over the work-group at once (one pair of barriers; each sum in
// the order of block_sum); red holds NV TB / 64 doubles
template <int NV>
__device__ inline void block_sum_n(double (&v)[NV], double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
#pragma unroll
    for (int c = 0; c < NV; ++c) v[c] += __shfl_xor(v[c], off);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int c = 0; c < NV; ++c) red[c * (TB / 64) + (threadIdx.x >> 6)] = v[c];
  }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NV; ++c) {
    double sc = 0.0;
#pragma unroll
    for (int k = 0; k < TB / 64; ++k) sc += red[c * (TB / 64) + k];
    v[c] = sc;
  }
}

// the NV components of the np partials (NV consecutive values per
// work-group), the same order in every work-group: thread t adds partials
// t, t + TB, ... (16-byte loads, issued together), then block_sum_n
template <int NV>
__device__ inline void sum_partials(const double* part, int np, double* red, double (&out)[NV]) {
  static_assert(NV % 2 == 0, "partials are read in pairs");
  const double2* p2 = reinterpret_cast<const double2*>(part);
#pragma unroll
  for (int c = 0; c < NV; ++c) out[c] = 0.0;
#pragma unroll 4
  for (int k = threadIdx.x; k < np; k += TB) {
#pragma unroll
    for (int c = 0; c < NV / 2; ++c) {
      const double2 x = p2[(size_t)k * (NV / 2) + c];
      out[2 * c] += x.x;
      out[2 * c + 1] += x.y;
    }
  }
  block_sum_n<NV>(out, red);
}

// Residual and scaled Jacobian of every cell; BiCGSTAB start vectors (x = 0,
// r = r^ = b); partials of |b|^2 into part[2], which bicg_first_kernel
// sums.
__global__ void __launch_bounds__(TB) assemble_kernel(TransportArgs a) {
  __shared__ double red[TB / 64];
  const int n = a.nx * a.ny;
  double bb = 0.0;
  for (int k = 0; k < CPT; ++k) {
    const int cell = (blockIdx.x * CPT + k) * TB + threadIdx.x;
    if (cell >= n) break;
    const int i = cell % a.nx, j = cell / a.nx;
    const double si = a.s[cell];
    const double fi = fw(si, a.M), dfi = fw_d1(si, a.M);
    // total volumetric fluxes through the four faces, +x / +y
    const double Fw = a.ux[(size_t)j * (a.nx + 1) + i] * a.hy;
    const double Fe = a.ux[(size_t)j * (a.nx + 1) + i + 1] * a.hy;
    const double Fs = a.uy[(size_t)j * a.nx + i] * a.hx;
    const double Fn = a.uy[(size_t)(j + 1) * a.nx + i] * a.hx;
    // net water outflow, d(outflow)/d(s_cell) and d(outflow)/d(s_neighbour)
    double out = 0.0, dg = 0.0, cw = 0.0, ce = 0.0, cs = 0.0, cn = 0.0;
    if (Fe > 0.0) {                // E face: leaves the cell
      out += fi * Fe; dg += dfi * Fe;
    } else if (i < a.nx - 1) {     // enters from the E neighbour
      const double sn = a.s[cell + 1];
      out += fw(sn, a.M) * Fe; ce = fw_d1(sn, a.M) * Fe;
    } else {                       // enters through the boundary
      out += a.fin * Fe;
    }
    if (Fn > 0.0) {
      out += fi * Fn; dg += dfi * Fn;
    } else if (j < a.ny - 1) {
      const double sn = a.s[cell + a.nx];
      out += fw(sn, a.M) * Fn; cn = fw_d1(sn, a.M) * Fn;
    } else {
      out += a.fin * Fn;
    }
    if (Fw < 0.0) {                // W face: a negative +x flux leaves the cell
      out -= fi * Fw; dg -= dfi * Fw;
    } else if (i > 0) {
      const double sn = a.s[cell - 1];
      out -= fw(sn, a.M) * Fw; cw = -fw_d1(sn, a.M) * Fw;
    } else {
      out -= a.fin * Fw;
    }
    if (Fs < 0.0) {
      out -= fi * Fs; dg -= dfi * Fs;
    } else if (j > 0) {
      const double sn = a.s[cell - a.nx];
      out -= fw(sn, a.M) * Fs; cs = -fw_d1(sn, a.M) * Fs;
    } else {
      out -= a.fin * Fs;
    }
    // wells: an injector adds water only, a producer removes the mixture
    double wsrc = 0.0;
    if (a.src) {
      const double qv = a.src[cell] * a.V;
      if (qv > 0.0) {
        wsrc = qv;
      } else if (qv < 0.0) {
        wsrc = qv * fi;
        dg -= qv * dfi;
      }
    }
    const double H = si - a.s_old[cell] + a.c * (out - wsrc);
    const double inv = 1.0 / (1.0 + a.c * dg);
    // the couplings, one per face (see TransportArgs::cfx): every face is
    // written by exactly one cell, the one whose row holds its coupling
    // (the downstream cell; for a face without flow, the cell on its +
    // side; a boundary face by its only cell, as 0)
    const size_t fx = (size_t)j * (a.nx + 1) + i, fy = (size_t)j * a.nx + i;
    if (Fw >= 0.0 || i == 0) a.cfx[fx] = i > 0 ? a.c * cw * inv : 0.0;
    if (Fe < 0.0 || i == a.nx - 1) a.cfx[fx + 1] = i < a.nx - 1 ? -(a.c * ce * inv) : 0.0;
    if (Fs >= 0.0 || j == 0) a.cfy[fy] = j > 0 ? a.c * cs * inv : 0.0;
    if (Fn < 0.0 || j == a.ny - 1) a.cfy[fy + a.nx] = j < a.ny - 1 ? -(a.c * cn * inv) : 0.0;
    const double bi = -H * inv;
    a.x[cell] = 0.0;
    a.r[cell] = bi;
    a.rh[cell] = bi;
    bb += bi * bi;
  }
  const double s = block_sum(bb, red);
  if (threadIdx.x == 0) {
    a.part[2][2 * (size_t)blockIdx.x + 0] = s;   // (r^, r) = |b|^2
    a.part[2][2 * (size_t)blockIdx.x + 1] = s;   // (r, r)
  }
}

// BiCGSTAB with two kernels (and two global reductions) per iteration.
// Kernel C of the textbook order (x += alpha p + omega q, r = q - omega t)
// is merged into the next iteration's kernel A (p = r + beta (p - omega v),
// v = A p): since r_{k+1} = q - omega t, the next rho = (r^, r_{k+1}) equals
// (r^, q) - omega (r^, t), which kernel B reduces with (t, q) and (t, t).
// |r|^2 for the convergence test is reduced from the r that is formed.
//
// Partials: part[0] (kernel A / AC -> B): (r^, v), (r, r); part[1]
// (B -> AC): (t, q), (t, t), (r^, q), (r^, t); part[2] (assembly): |b|^2.

// Iteration 0's kernel A: rho_0 = (r^, r_0) = |b|^2 from the assembly's
// partials, p_0 = r_0, v_0 = A p_0; partials (r^, v_0), (r_0, r_0).
// It also sets the solve's start state (the flag of the previous solve is
// not read).
__global__ void __launch_bounds__(TB) bicg_first_kernel(TransportArgs a, int np) {
  __shared__ double red[2 * TB / 64];
  double sb[2];
  sum_partials<2>(a.part[2], np, red, sb);
  const double bb = sb[0];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.scal[TS_BB] = bb;
    a.scal[TS_DONE] = bb > 0.0 ? 0.0 : 1.0;   // H = 0: nothing to solve
    a.scal[TS_ITERS] = 0.0;
    a.scal[TS_RR] = bb;
    a.scal[TS_RHO + 0] = bb;
  }
  double* pn = a.p[0];
  double* vn = a.v[0];
  const int n = a.nx * a.ny;
  // the loads of all CPT cells are issued together: indices are clamped
  // rather than branched on, the terms of missing neighbours are dropped by
  // selects (in the stencil's order of addition), and the stores wait until
  // every value is formed
  double pcs[CPT], vvs[CPT];
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < CPT; ++kk) {
    const int cell = (blockIdx.x * CPT + kk) * TB + threadIdx.x;
    const int cc = min(cell, n - 1);
    const int i = cc % a.nx, j = cc / a.nx;
    const int cw = i > 0 ? cc - 1 : cc, ce = i < a.nx - 1 ? cc + 1 : cc;
    const int cs = j > 0 ? cc - a.nx : cc, cn = j < a.ny - 1 ? cc + a.nx : cc;
    const size_t fx = (size_t)j * (a.nx + 1) + i, fy = (size_t)j * a.nx + i;
    const double w = fmin(a.cfx[fx], 0.0), e = -fmax(a.cfx[fx + 1], 0.0);
    const double so = fmin(a.cfy[fy], 0.0), no = -fmax(a.cfy[fy + a.nx], 0.0);
    const double rh = a.rh[cc];
    const double pc = a.r[cc], pw = a.r[cw], pe = a.r[ce], ps = a.r[cs], pnb = a.r[cn];
    double vv = pc;
    vv += i > 0 ? w * pw : 0.0;
    vv += i < a.nx - 1 ? e * pe : 0.0;
    vv += j > 0 ? so * ps : 0.0;
    vv += j < a.ny - 1 ? no * pnb : 0.0;
    pcs[kk] = pc;
    vvs[kk] = vv;
    if (cell < n) {
      acc[0] += rh * vv;
      acc[1] += pc * pc;
    }
  }
#pragma unroll
  for (int kk = 0; kk < CPT; ++kk) {
    const int cell = (blockIdx.x * CPT + kk) * TB + threadIdx.x;
    if (cell < n) {
      pn[cell] = pcs[kk];
      vn[cell] = vvs[kk];
    }
  }
  block_sum_n<2>(acc, red);
  if (threadIdx.x == 0) {
    a.part[0][2 * (size_t)blockIdx.x + 0] = acc[0];
    a.part[0][2 * (size_t)blockIdx.x + 1] = acc[1];
  }
}

// Kernel B of iteration k (par = k & 1): the stopping tests on r_k
// (converged; breakdown: omega_{k-1} = 0, rho_k = 0 or not finite, (r^, v_k)
// = 0; iteration limit); alpha = rho_k / (r^, v_k); q = r - alpha v (the "s"
// of BiCGSTAB) and t = A q (neighbours' q on the fly); partials (t, q),
// (t, t), (r^, q), (r^, t).
__global__ void __launch_bounds__(TB) bicg_b_kernel(TransportArgs a, int k, int np) {
  __shared__ double red[4 * TB / 64];
  if (a.scal[TS_DONE] != 0.0) return;
  const int par = k & 1, prv = par ^ 1;
  double sv[2];
  sum_partials<2>(a.part[0], np, red, sv);
  const double rv = sv[0], rr = sv[1];
  const double rho = a.scal[TS_RHO + par];
  const bool conv = rr <= a.tol2 * a.scal[TS_BB];
  // omega_{k-1} = 0 with r_k != 0 stalls BiCGSTAB
  const bool brk = (k > 0 && !(a.scal[TS_OMEGA + prv] != 0.0)) || !(rho != 0.0) || !isfinite(rho);
  if (conv || brk || k >= a.max_iter) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.scal[TS_DONE] = conv ? 1.0 : 2.0;
      a.scal[TS_ITERS] = k;
      a.scal[TS_RR] = rr;
    }
    return;
  }
  const double alpha = rho / rv;
  if (!(rv != 0.0) || !isfinite(alpha)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.scal[TS_DONE] = 2.0;
      a.scal[TS_ITERS] = k;
      a.scal[TS_RR] = rr;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.scal[TS_ALPHA + par] = alpha;
  const double* vn = a.v[par];
  const int n = a.nx * a.ny;
  // loads of all CPT cells issued together, as in bicg_first_kernel
  double qcs[CPT], tvs[CPT];
  double acc[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < CPT; ++kk) {
    const int cell = (blockIdx.x * CPT + kk) * TB + threadIdx.x;
    const int cc = min(cell, n - 1);
    const int i = cc % a.nx, j = cc / a.nx;
    const int cw = i > 0 ? cc - 1 : cc, ce = i < a.nx - 1 ? cc + 1 : cc;
    const int cs = j > 0 ? cc - a.nx : cc, cn = j < a.ny - 1 ? cc + a.nx : cc;
    auto qnew = [&](int c2) {
      const double r = a.r[c2], v = vn[c2];
      return r - alpha * v;
    };
    const size_t fx = (size_t)j * (a.nx + 1) + i, fy = (size_t)j * a.nx + i;
    const double w = fmin(a.cfx[fx], 0.0), e = -fmax(a.cfx[fx + 1], 0.0);
    const double so = fmin(a.cfy[fy], 0.0), no = -fmax(a.cfy[fy + a.nx], 0.0);
    const double rh = a.rh[cc];
    const double qc = qnew(cc), qw = qnew(cw), qe = qnew(ce), qs = qnew(cs), qn = qnew(cn);
    double tv = qc;
    tv += i > 0 ? w * qw : 0.0;
    tv += i < a.nx - 1 ? e * qe : 0.0;
    tv += j > 0 ? so * qs : 0.0;
    tv += j < a.ny - 1 ? no * qn : 0.0;
    qcs[kk] = qc;
    tvs[kk] = tv;
    if (cell < n) {
      acc[0] += tv * qc;
      acc[1] += tv * tv;
      acc[2] += rh * qc;
      acc[3] += rh * tv;
    }
  }
#pragma unroll
  for (int kk = 0; kk < CPT; ++kk) {
    const int cell = (blockIdx.x * CPT + kk) * TB + threadIdx.x;
    if (cell < n) {
      a.q[cell] = qcs[kk];
      a.t[cell] = tvs[kk];
    }
  }
  block_sum_n<4>(acc, red);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int c = 0; c < 4; ++c) a.part[1][4 * (size_t)blockIdx.x + c] = acc[c];
  }
}

// Kernel AC of iteration k (par = k & 1, nxt = par ^ 1): omega_k =
// (t, q) / (t, t); x += alpha p_k + omega q; r_{k+1} = q - omega t;
// rho_{k+1} = (r^, q) - omega (r^, t), beta = (rho_{k+1} / rho_k)
// (alpha / omega); p_{k+1} = r_{k+1} + beta (p_k - omega v_k) and
// v_{k+1} = A p_{k+1} (the neighbours' r and p formed on the fly);
// partials (r^, v_{k+1}), (r_{k+1}, r_{k+1}).  A breakdown here (omega = 0,
// rho_{k+1} = 0) leaves p and v meaningless; the next kernel B stops on it.
__global__ void __launch_bounds__(TB) bicg_ac_kernel(TransportArgs a, int k, int np) {
  __shared__ double red[4 * TB / 64];
  if (a.scal[TS_DONE] != 0.0) return;
  const int par = k & 1, nxt = par ^ 1;
  double sb[4];
  sum_partials<4>(a.part[1], np, red, sb);
  const double tq = sb[0], tt = sb[1], rq = sb[2], rt = sb[3];
  const double alpha = a.scal[TS_ALPHA + par];
  // t = 0 means q = 0: the half step already solved the system
  const double omega = tt > 0.0 ? tq / tt : 0.0;
  const double rho1 = rq - omega * rt;
  const double beta = (rho1 / a.scal[TS_RHO + par]) * (alpha / omega);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.scal[TS_OMEGA + par] = omega;
    a.scal[TS_RHO + nxt] = rho1;
  }
  const double* po = a.p[par];
  const double* vo = a.v[par];
  double* pn = a.p[nxt];
  double* vn = a.v[nxt];
  const int n = a.nx * a.ny;
  // loads of all CPT cells issued together, as in bicg_first_kernel
  double xs[CPT], rcs[CPT], pcs[CPT], vvs[CPT];
  double acc[2] = {0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < CPT; ++kk) {
    const int cell = (blockIdx.x * CPT + kk) * TB + threadIdx.x;
    const int cc = min(cell, n - 1);
    const int i = cc % a.nx, j = cc / a.nx;
    const int cw = i > 0 ? cc - 1 : cc, ce = i < a.nx - 1 ? cc + 1 : cc;
    const int cs = j > 0 ? cc - a.nx : cc, cn = j < a.ny - 1 ? cc + a.nx : cc;
    auto rnew = [&](int c2) {
      const double q = a.q[c2], t = a.t[c2];
      return q - omega * t;
    };
    auto pnew = [&](int c2, double r) {
      const double pv = po[c2], v = vo[c2];
      return r + beta * (pv - omega * v);
    };
    const size_t fx = (size_t)j * (a.nx + 1) + i, fy = (size_t)j * a.nx + i;
    const double w = fmin(a.cfx[fx], 0.0), e = -fmax(a.cfx[fx + 1], 0.0);
    const double so = fmin(a.cfy[fy], 0.0), no = -fmax(a.cfy[fy + a.nx], 0.0);
    const double rh = a.rh[cc];
    const double xo = a.x[cc], qo = a.q[cc], pk = po[cc];
    const double rc = rnew(cc);
    const double pc = pnew(cc, rc), pw = pnew(cw, rnew(cw)), pe = pnew(ce, rnew(ce));
    const double ps = pnew(cs, rnew(cs)), pnb = pnew(cn, rnew(cn));
    double vv = pc;
    vv += i > 0 ? w * pw : 0.0;
    vv += i < a.nx - 1 ? e * pe : 0.0;
    vv += j > 0 ? so * ps : 0.0;
    vv += j < a.ny - 1 ? no * pnb : 0.0;
    xs[kk] = xo + (alpha * pk + omega * qo);
    rcs[kk] = rc;
    pcs[kk] = pc;
    vvs[kk] = vv;
    if (cell < n) {
      acc[0] += rh * vv;
      acc[1] += rc * rc;
    }
  }
#pragma unroll
  for (int kk = 0; kk < CPT; ++kk) {
    const int cell = (blockIdx.x * CPT + kk) * TB + threadIdx.x;
    if (cell < n) {
      a.x[cell] = xs[kk];
      a.r[cell] = rcs[kk];
      pn[cell] = pcs[kk];
      vn[cell] = vvs[kk];
    }
  }
  block_sum_n<2>(acc, red);
  if (threadIdx.x == 0) {
    a.part[0][2 * (size_t)blockIdx.x + 0] = acc[0];
    a.part[0][2 * (size_t)blockIdx.x + 1] = acc[1];
  }
}

// Newton update with the bound and the inflection-point rule; partials of
// V (s_new - s)^2 into part[0]
__global__ void __launch_bounds__(TB) update_kernel(TransportArgs a) {
  __shared__ double red[TB / 64];
  // queued after every BiCGSTAB batch: applies the direction only once the
  // solve has stopped
  if (a.scal[TS_DONE] == 0.0) return;
  const int n = a.nx * a.ny;
  double ch = 0.0;
  for (int k = 0; k < CPT; ++k) {
    const int cell = (blockIdx.x * CPT + k) * TB + threadIdx.x;
    if (cell >= n) break;
    const double s = a.s[cell];
    double sn = fmin(fmax(s + a.x[cell], 0.0), 1.0);
    if (fw_d2_sign(sn, a.M) * fw_d2_sign(s, a.M) < 0) sn = 0.5 * (sn + s);
    a.s[cell] = sn;
    ch += (sn - s) * (sn - s);
  }
  const double s = block_sum(ch, red);
  if (threadIdx.x == 0) {
    a.part[0][2 * (size_t)blockIdx.x + 0] = s;
    a.part[0][2 * (size_t)blockIdx.x + 1] = 0.0;
  }
}

__global__ void __launch_bounds__(TB) change_kernel(TransportArgs a, int np) {
  __shared__ double red[2 * TB / 64];
  if (a.scal[TS_DONE] == 0.0) return;
  double sc[2];
  sum_partials<2>(a.part[0], np, red, sc);
  const double ch = sc[0];
  if (threadIdx.x == 0) a.scal[TS_CHANGE] = ch * a.V;
}

// max |a - b| over the cells: per-work-group maxima into part[0], then one
// work-group reduces them (fixed order) into scal[TS_OUTER]
__global__ void __launch_bounds__(TB) maxdiff_kernel(TransportArgs t, const double* a, const double* b) {
  __shared__ double red[TB / 64];
  const int n = t.nx * t.ny;
  double m = 0.0;
  for (int k = 0; k < CPT; ++k) {
    const int cell = (blockIdx.x * CPT + k) * TB + threadIdx.x;
    if (cell >= n) break;
    m = fmax(m, fabs(a[cell] - b[cell]));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int k = 0; k < TB / 64; ++k) r = fmax(r, red[k]);
    t.part[0][2 * (size_t)blockIdx.x] = r;
  }
}

__global__ void __launch_bounds__(TB) maxdiff_reduce_kernel(TransportArgs t, int np) {
  __shared__ double red[TB / 64];
  double m = 0.0;
  for (int k = threadIdx.x; k < np; k += TB) m = fmax(m, t.part[0][2 * (size_t)k]);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int k = 0; k < TB / 64; ++k) r = fmax(r, red[k]);
    t.scal[TS_OUTER] = r;
  }
}

__global__ void copy_kernel(double* dst, const double* src, size_t n) {
  for (size_t i = blockIdx.x * (size_t)blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    dst[i] = src[i];
}

}  // namespace

int transport_blocks(int nx, int ny) {
  const long long n = (long long)nx * ny;
  return (int)((n + (long long)TB * CPT - 1) / ((long long)TB * CPT));
}

hipError_t launch_transport_assemble(const TransportArgs& a, hipStream_t st) {
  const int nb = transport_blocks(a.nx, a.ny);
  hipLaunchKernelGGL(assemble_kernel, dim3(nb), dim3(TB), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_transport_bicg(const TransportArgs& a, int k0, int count, hipStream_t st) {
  const int nb = transport_blocks(a.nx, a.ny);
  for (int k = k0; k < k0 + count; ++k) {
    if (k == 0) hipLaunchKernelGGL(bicg_first_kernel, dim3(nb), dim3(TB), 0, st, a, nb);
    hipLaunchKernelGGL(bicg_b_kernel, dim3(nb), dim3(TB), 0, st, a, k, nb);
    hipLaunchKernelGGL(bicg_ac_kernel, dim3(nb), dim3(TB), 0, st, a, k, nb);
  }
  return hipGetLastError();
}

hipError_t launch_transport_update(const TransportArgs& a, hipStream_t st) {
  const int nb = transport_blocks(a.nx, a.ny);
  hipLaunchKernelGGL(update_kernel, dim3(nb), dim3(TB), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(change_kernel, dim3(1), dim3(TB), 0, st, a, nb);
  return hipGetLastError();
}

hipError_t launch_transport_maxdiff(const TransportArgs& t, const double* a, const double* b,
                                   hipStream_t st) {
  const int nb = transport_blocks(t.nx, t.ny);
  hipLaunchKernelGGL(maxdiff_kernel, dim3(nb), dim3(TB), 0, st, t, a, b);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(maxdiff_reduce_kernel, dim3(1), dim3(TB), 0, st, t, nb);
  return hipGetLastError();
}

hipError_t launch_copy(double* dst, const double* src, size_t n, hipStream_t st) {
  hipLaunchKernelGGL(copy_kernel, dim3(1024), dim3(256), 0, st, dst, src, n);
  return hipGetLastError();
}

}  // namespace mrcm
