// Implicit transport of the water saturation (paper, section 4) on the GPU:
// implicit Euler with first-order upwind fluxes (eqs. (BL2D_Newton2),
// (fluxes_impli), (up_fluxes_impli)), Newton's method (eqs. (BL2D_Newton8),
// (BL2D_Newton7)) with the inflection-point strategy, one cell per thread.
//
// Per Newton iteration:
//  * assemble_kernel: the residual H and the Jacobian H' of every cell.  A
//    face's water flux depends on the saturation of its upwind cell only, so
//    a cell's row couples it to the neighbours its water comes from.  Rows
//    are scaled by their diagonal (Jacobi), which leaves a unit diagonal,
//    four coupling coefficients and the right-hand side -H / diag.
//  * BiCGSTAB on the scaled system, three fused kernels per iteration (p and
//    v = A p; s and t = A s; x, r), each forming the neighbours' values it
//    needs from the previous vectors instead of a separate pass.  Inner
//    products are reduced per work-group into partial sums that the next
//    kernel's work-groups all sum in the same fixed order (deterministic, no
//    atomics), so every work-group forms the iteration's scalars itself.
//    Convergence or breakdown sets a flag in device memory that makes the
//    remaining launches of a batch return at once.
//  * update_kernel: s <- clamp(s + d) to [0, 1], then the inflection-point
//    rule (an update whose ends lie on different sides of the inflection
//    point of f is halved), and the partial sums of the change's squared
//    L2 norm.
//
// Layout: cell (i, j) at j*nx + i; face velocities as the Darcy step
// returns them (ux on (nx+1)*ny x-faces, uy on nx*(ny+1) y-faces).
#include "mrcm_internal.h"

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

// two sums over the work-group at once (one pair of barriers; each sum in
// the order of block_sum); red holds 2 TB / 64 doubles
__device__ inline double2 block_sum2(double u, double v, double* red) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    u += __shfl_xor(u, off);
    v += __shfl_xor(v, off);
  }
  __syncthreads();
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = u;
    red[TB / 64 + (threadIdx.x >> 6)] = v;
  }
  __syncthreads();
  double su = 0.0, sv = 0.0;
#pragma unroll
  for (int k = 0; k < TB / 64; ++k) {
    su += red[k];
    sv += red[TB / 64 + k];
  }
  return make_double2(su, sv);
}

// both components of the np partials (pairs), the same order in every
// work-group: thread t adds partials t, t + TB, ... (16-byte loads, issued
// together), then block_sum2
__device__ inline double2 sum_partials(const double* part, int np, double* red) {
  const double2* p2 = reinterpret_cast<const double2*>(part);
  double u = 0.0, v = 0.0;
#pragma unroll 4
  for (int k = threadIdx.x; k < np; k += TB) {
    const double2 x = p2[k];
    u += x.x;
    v += x.y;
  }
  return block_sum2(u, v, red);
}



// Residual and scaled Jacobian of every cell; BiCGSTAB start (x = 0,
// r = r^ = b, p = v = 0); partials of |b|^2 into part[2] (read as the
// "previous kernel C" by the first iteration).
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
    a.aw[cell] = a.c * cw * inv;
    a.ae[cell] = a.c * ce * inv;
    a.as[cell] = a.c * cs * inv;
    a.an[cell] = a.c * cn * inv;
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

// Kernel A of iteration k (par = k & 1): rho_k = (r^, r_k) and |r_k|^2 from
// kernel C's partials; convergence check; p_k = r + beta (p_{k-1} - omega
// v_{k-1}) and v_k = A p_k (neighbours' p formed on the fly); partials of
// (r^, v_k).
// FIRST: iteration 0, whose p is r (the previous p and v hold nothing and
// are not read)
template <bool FIRST>
__global__ void __launch_bounds__(TB) bicg_a_kernel(TransportArgs a, int k, int np) {
  __shared__ double red[2 * TB / 64];
  if (a.scal[TS_DONE] != 0.0) return;
  const int par = k & 1, prv = par ^ 1;
  const double2 sr = sum_partials(a.part[2], np, red);
  const double rho = sr.x, rr = sr.y;
  const double bb = a.scal[TS_BB];
  const bool conv = rr <= a.tol2 * bb;
  const bool brk = !(rho != 0.0) || !isfinite(rho);
  if (conv || brk || k >= a.max_iter) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.scal[TS_DONE] = conv ? 1.0 : 2.0;
      a.scal[TS_ITERS] = k;
      a.scal[TS_RR] = rr;
    }
    return;
  }
  const double beta = FIRST ? 0.0 : (rho / a.scal[TS_RHO + prv]) * (a.scal[TS_ALPHA + prv] / a.scal[TS_OMEGA + prv]);
  const double om = FIRST ? 0.0 : a.scal[TS_OMEGA + prv];
  if (blockIdx.x == 0 && threadIdx.x == 0) a.scal[TS_RHO + par] = rho;
  const double* po = a.p[prv];
  const double* vo = a.v[prv];
  double* pn = a.p[par];
  double* vn = a.v[par];
  const int n = a.nx * a.ny;
  // the loads of all CPT cells are issued together: indices are clamped
  // rather than branched on, the terms of missing neighbours are dropped by
  // selects (in the stencil's order of addition), and the stores wait until
  // every value is formed
  double pcs[CPT], vvs[CPT];
  double rv = 0.0;
#pragma unroll
  for (int kk = 0; kk < CPT; ++kk) {
    const int cell = (blockIdx.x * CPT + kk) * TB + threadIdx.x;
    const int cc = min(cell, n - 1);
    const int i = cc % a.nx, j = cc / a.nx;
    const int cw = i > 0 ? cc - 1 : cc, ce = i < a.nx - 1 ? cc + 1 : cc;
    const int cs = j > 0 ? cc - a.nx : cc, cn = j < a.ny - 1 ? cc + a.nx : cc;
    auto pnew = [&](int c2) {
      if (FIRST) return a.r[c2];
      const double r = a.r[c2], pv = po[c2], v = vo[c2];
      return r + beta * (pv - om * v);
    };
    const double w = a.aw[cc], e = a.ae[cc], so = a.as[cc], no = a.an[cc], rh = a.rh[cc];
    const double pc = pnew(cc), pw = pnew(cw), pe = pnew(ce), ps = pnew(cs), pnb = pnew(cn);
    double vv = pc;
    vv += i > 0 ? w * pw : 0.0;
    vv += i < a.nx - 1 ? e * pe : 0.0;
    vv += j > 0 ? so * ps : 0.0;
    vv += j < a.ny - 1 ? no * pnb : 0.0;
    pcs[kk] = pc;
    vvs[kk] = vv;
    if (cell < n) rv += rh * vv;
  }
#pragma unroll
  for (int kk = 0; kk < CPT; ++kk) {
    const int cell = (blockIdx.x * CPT + kk) * TB + threadIdx.x;
    if (cell < n) {
      pn[cell] = pcs[kk];
      vn[cell] = vvs[kk];
    }
  }
  const double s = block_sum(rv, red);
  if (threadIdx.x == 0) {
    a.part[0][2 * (size_t)blockIdx.x + 0] = s;
    a.part[0][2 * (size_t)blockIdx.x + 1] = 0.0;
  }
}

// Kernel B: alpha = rho / (r^, v); q = r - alpha v (the "s" of BiCGSTAB)
// and t = A q (neighbours' q on the fly); partials of (t, q), (t, t).
__global__ void __launch_bounds__(TB) bicg_b_kernel(TransportArgs a, int k, int np) {
  __shared__ double red[2 * TB / 64];
  if (a.scal[TS_DONE] != 0.0) return;
  const int par = k & 1;
  const double rv = sum_partials(a.part[0], np, red).x;
  const double alpha = a.scal[TS_RHO + par] / rv;
  if (!(rv != 0.0) || !isfinite(alpha)) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      a.scal[TS_DONE] = 2.0;
      a.scal[TS_ITERS] = k;
    }
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) a.scal[TS_ALPHA + par] = alpha;
  const double* vn = a.v[par];
  const int n = a.nx * a.ny;
  // loads of all CPT cells issued together, as in kernel A
  double qcs[CPT], tvs[CPT];
  double ts = 0.0, tt = 0.0;
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
    const double w = a.aw[cc], e = a.ae[cc], so = a.as[cc], no = a.an[cc];
    const double qc = qnew(cc), qw = qnew(cw), qe = qnew(ce), qs = qnew(cs), qn = qnew(cn);
    double tv = qc;
    tv += i > 0 ? w * qw : 0.0;
    tv += i < a.nx - 1 ? e * qe : 0.0;
    tv += j > 0 ? so * qs : 0.0;
    tv += j < a.ny - 1 ? no * qn : 0.0;
    qcs[kk] = qc;
    tvs[kk] = tv;
    if (cell < n) {
      ts += tv * qc;
      tt += tv * tv;
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
  const double2 s = block_sum2(ts, tt, red);
  if (threadIdx.x == 0) {
    a.part[1][2 * (size_t)blockIdx.x + 0] = s.x;
    a.part[1][2 * (size_t)blockIdx.x + 1] = s.y;
  }
}

// Kernel C: omega = (t, q) / (t, t); x += alpha p + omega q; r = q - omega t;
// partials of (r^, r), (r, r) for the next kernel A.
__global__ void __launch_bounds__(TB) bicg_c_kernel(TransportArgs a, int k, int np) {
  __shared__ double red[2 * TB / 64];
  if (a.scal[TS_DONE] != 0.0) return;
  const int par = k & 1;
  const double2 st = sum_partials(a.part[1], np, red);
  const double ts = st.x, tt = st.y;
  const double alpha = a.scal[TS_ALPHA + par];
  // t = 0 means q = 0: the half step already solved the system
  const double omega = tt > 0.0 ? ts / tt : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) a.scal[TS_OMEGA + par] = omega;
  const double* pn = a.p[par];
  const int n = a.nx * a.ny;
  // loads of all CPT cells issued together, as in kernel A
  double xs[CPT], rcs[CPT];
  double rhr = 0.0, rr = 0.0;
#pragma unroll
  for (int kk = 0; kk < CPT; ++kk) {
    const int cell = (blockIdx.x * CPT + kk) * TB + threadIdx.x;
    const int cc = min(cell, n - 1);
    const double qc = a.q[cc], xo = a.x[cc], pc = pn[cc], tc = a.t[cc], rh = a.rh[cc];
    xs[kk] = xo + (alpha * pc + omega * qc);
    const double rc = qc - omega * tc;
    rcs[kk] = rc;
    if (cell < n) {
      rhr += rh * rc;
      rr += rc * rc;
    }
  }
#pragma unroll
  for (int kk = 0; kk < CPT; ++kk) {
    const int cell = (blockIdx.x * CPT + kk) * TB + threadIdx.x;
    if (cell < n) {
      a.x[cell] = xs[kk];
      a.r[cell] = rcs[kk];
    }
  }
  const double2 s = block_sum2(rhr, rr, red);
  if (threadIdx.x == 0) {
    a.part[2][2 * (size_t)blockIdx.x + 0] = s.x;
    a.part[2][2 * (size_t)blockIdx.x + 1] = s.y;
  }
  // omega = 0 with t != 0 stalls BiCGSTAB: stop (breakdown)
  if (!(omega != 0.0) && tt > 0.0 && blockIdx.x == 0 && threadIdx.x == 0) {
    a.scal[TS_DONE] = 2.0;
    a.scal[TS_ITERS] = k + 1;
  }
}

// |b|^2 from the assembly's partials, and the solve's start state
__global__ void __launch_bounds__(TB) bicg_start_kernel(TransportArgs a, int np) {
  __shared__ double red[2 * TB / 64];
  const double bb = sum_partials(a.part[2], np, red).x;
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    a.scal[TS_BB] = bb;
    a.scal[TS_DONE] = bb > 0.0 ? 0.0 : 1.0;   // H = 0: nothing to solve
    a.scal[TS_ITERS] = 0.0;
    a.scal[TS_RR] = bb;
  }
}

// Newton update with the bound and the inflection-point rule; partials of
// V (s_new - s)^2 into part[0]
__global__ void __launch_bounds__(TB) update_kernel(TransportArgs a) {
  __shared__ double red[TB / 64];
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
  const double ch = sum_partials(a.part[0], np, red).x;
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
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(bicg_start_kernel, dim3(1), dim3(TB), 0, st, a, nb);
  return hipGetLastError();
}

hipError_t launch_transport_bicg(const TransportArgs& a, int k0, int count, hipStream_t st) {
  const int nb = transport_blocks(a.nx, a.ny);
  for (int k = k0; k < k0 + count; ++k) {
    if (k == 0)
      hipLaunchKernelGGL(bicg_a_kernel<true>, dim3(nb), dim3(TB), 0, st, a, k, nb);
    else
      hipLaunchKernelGGL(bicg_a_kernel<false>, dim3(nb), dim3(TB), 0, st, a, k, nb);
    hipLaunchKernelGGL(bicg_b_kernel, dim3(nb), dim3(TB), 0, st, a, k, nb);
    hipLaunchKernelGGL(bicg_c_kernel, dim3(nb), dim3(TB), 0, st, a, k, nb);
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
