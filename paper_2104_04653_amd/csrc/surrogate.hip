// Learned surrogate of the local basis functions: a 4-layer 3x3
// convolutional network in BF16 with FP32 accumulation on the matrix cores
// (v_mfma_f32_16x16x16bf16_1k), with hand-written forward, backward and Adam
// kernels (gfx950).
//
// Input of one subdomain: 5 channels on its 16 x 16 cells, stored
// channels-last (pixel-major, channel padded to 8): the normalised log
// mobility-permeability z = (ln kappa - mean ln kappa) / 4 and four masks that
// mark the cells next to each side (W, E, S, N) whose face lies on the
// skeleton.  Output: the 16 basis functions of the subdomain (columns of
// the W, E, S, N interface dofs, see local_mfma.hip) in a normalised form:
// pressure-dof columns as they are, flux-dof columns times
// kappa_g / (alpha H) with kappa_g the geometric mean of kappa over the
// subdomain.  Scaling kappa by a constant leaves the pressure columns
// unchanged and divides the flux columns by it (the Robin data of a flux
// dof is T_R beta = |f| alpha H / (d + alpha H), independent of kappa), so
// both normalised columns are scale-free.
//
// Layers: 5(8) -> 32 -> 32 -> 32 -> 16, ReLU after the first three.  A
// convolution is a GEMM with M = output channels, N = the 256 pixels (16
// MFMA tiles, one image row each) and K = 9 taps x input channels ordered
// (tap, channel), so that the four K values a lane supplies are four
// consecutive channels of one shifted pixel: one 8-byte LDS read.  The
// lane layout of the BF16 MFMA (A[i][k]: lane i + 16 (k/4), element k%4;
// B[k][j]: lane j + 16 (k/4); D[i][j]: lane j + 16 (i/4), element i%4) was
// checked on the device.
#include "mrcm_internal.h"

#include <math.h>

namespace mrcm {
namespace cnn {

typedef short s4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

constexpr int NLAYERS = 4;
constexpr int NPIX = 256;
constexpr int HW = 16;
constexpr int HALO = 18;
constexpr int NT = 256;

__device__ inline short f2bf(float x) {
  unsigned u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);   // round to nearest even
  return (short)(u >> 16);
}
__device__ inline float bf2f(short b) { return __uint_as_float(((unsigned)(unsigned short)b) << 16); }

__device__ inline f4 mma(s4 a, s4 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

template <int C>
constexpr int kpad() { return (9 * C + 15) / 16 * 16; }

// load one patch (NPIX x C, channels-last) into an LDS tile with a zero halo
template <int C>
__device__ void load_halo(const short* src, short* Xs) {
  static_assert(C % 4 == 0, "four channels per 8-byte move");
  s4* X4 = reinterpret_cast<s4*>(Xs);
  const s4* S4 = reinterpret_cast<const s4*>(src);
  for (int e = threadIdx.x; e < HALO * HALO * C / 4; e += NT) X4[e] = s4{0, 0, 0, 0};
  __syncthreads();
  for (int e = threadIdx.x; e < NPIX * C / 4; e += NT) {
    const int p = e / (C / 4), c4 = e % (C / 4);
    X4[((p / HW + 1) * HALO + p % HW + 1) * (C / 4) + c4] = S4[e];
  }
}

// ---------------------------------------------------------------------------
// forward: out[p][co] = act(sum_{tap,ci} W[co][tap][ci] x[p + off(tap)][ci] + b[co])
// ---------------------------------------------------------------------------
template <int CIN, int COUT, bool RELU, bool OUTF32>
__global__ void __launch_bounds__(NT) conv_fwd_kernel(const short* in, const short* W,
                                                      const float* bias, short* out_bf,
                                                      float* out_f) {
  // Each wave keeps the weight fragments of all output-channel tiles in
  // registers (read once from the LDS copy of the weights), reads each
  // input fragment once from LDS for all of them, and stores four
  // consecutive channels of a pixel per lane in one write.
  constexpr int KP = kpad<CIN>(), NK = KP / 16, MT = COUT / 16;
  __shared__ __attribute__((aligned(16))) short Xs[HALO * HALO * CIN];
  __shared__ __attribute__((aligned(16))) short Ws[COUT * KP];
  const int b = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = lane & 15, g = lane >> 4;
  for (int e = threadIdx.x; e < COUT * KP / 4; e += NT)   // coalesced 8-byte copies
    reinterpret_cast<s4*>(Ws)[e] = reinterpret_cast<const s4*>(W)[e];
  load_halo<CIN>(in + (size_t)b * NPIX * CIN, Xs);
  float bv4[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) bv4[mt][v] = bias[mt * 16 + 4 * g + v];
  __syncthreads();
  s4 av[MT][NK];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int kk = 0; kk < NK; ++kk)
      av[mt][kk] = *reinterpret_cast<const s4*>(&Ws[(mt * 16 + x) * KP + 16 * kk + 4 * g]);
  for (int yy = 0; yy < 4; ++yy) {
    const int y = wv * 4 + yy;
    f4 acc[MT];
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < NK; ++kk) {
      const int k0 = 16 * kk + 4 * g, tap = k0 / CIN, ci = k0 % CIN;
      s4 bv = {0, 0, 0, 0};
      if (tap < 9) {
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        bv = *reinterpret_cast<const s4*>(&Xs[((y + dy + 1) * HALO + x + dx + 1) * CIN + ci]);
      }
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[mt] = mma(av[mt][kk], bv, acc[mt]);
    }
    const size_t p = (size_t)b * NPIX + y * HW + x;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      float val[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        val[v] = acc[mt][v] + bv4[mt][v];
        if (RELU) val[v] = fmaxf(val[v], 0.f);
      }
      const int co = mt * 16 + 4 * g;
      if (OUTF32) {
        *reinterpret_cast<f4*>(&out_f[p * COUT + co]) = f4{val[0], val[1], val[2], val[3]};
      } else {
        *reinterpret_cast<s4*>(&out_bf[p * COUT + co]) =
            s4{f2bf(val[0]), f2bf(val[1]), f2bf(val[2]), f2bf(val[3])};
      }
    }
  }
}

// ---------------------------------------------------------------------------
// inference: the four layers of one patch in one work-group, the
// activations kept in LDS (two 32-channel tiles with a zero halo, used in
// turn; the 8-channel input has a tile of its own).  The arithmetic is the
// per-layer kernel's (same K order, same BF16 rounding of the activations),
// so the outputs are the same bits, without the three activation round
// trips through HBM and three launches.
// ---------------------------------------------------------------------------
template <int CIN, int COUT, bool RELU, bool OUTF32>
__device__ void conv_layer_lds(const short* Xin, const short* W, const float* bias, short* Ws,
                               short* Xout, float* out_f) {
  constexpr int KP = kpad<CIN>(), NK = KP / 16, MT = COUT / 16;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = lane & 15, g = lane >> 4;
  for (int e = threadIdx.x; e < COUT * KP / 4; e += NT)   // coalesced 8-byte copies
    reinterpret_cast<s4*>(Ws)[e] = reinterpret_cast<const s4*>(W)[e];
  float bv4[MT][4];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int v = 0; v < 4; ++v) bv4[mt][v] = bias[mt * 16 + 4 * g + v];
  __syncthreads();   // weights staged; the input tile is complete
  s4 av[MT][NK];
#pragma unroll
  for (int mt = 0; mt < MT; ++mt)
#pragma unroll
    for (int kk = 0; kk < NK; ++kk)
      av[mt][kk] = *reinterpret_cast<const s4*>(&Ws[(mt * 16 + x) * KP + 16 * kk + 4 * g]);
  // the wave's four image rows at once: eight independent accumulators
  // keep the matrix cores busy (one row at a time waits on each MFMA)
  f4 acc[4][MT];
#pragma unroll
  for (int yy = 0; yy < 4; ++yy)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[yy][mt] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int kk = 0; kk < NK; ++kk) {
    const int k0 = 16 * kk + 4 * g, tap = k0 / CIN, ci = k0 % CIN;
    const int dy = tap / 3 - 1, dx = tap % 3 - 1;
    s4 bv[4];
#pragma unroll
    for (int yy = 0; yy < 4; ++yy) {
      const int y = wv * 4 + yy;
      bv[yy] = s4{0, 0, 0, 0};
      if (tap < 9) bv[yy] = *reinterpret_cast<const s4*>(&Xin[((y + dy + 1) * HALO + x + dx + 1) * CIN + ci]);
    }
#pragma unroll
    for (int yy = 0; yy < 4; ++yy)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt) acc[yy][mt] = mma(av[mt][kk], bv[yy], acc[yy][mt]);
  }
#pragma unroll
  for (int yy = 0; yy < 4; ++yy) {
    const int y = wv * 4 + yy;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      float val[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        val[v] = acc[yy][mt][v] + bv4[mt][v];
        if (RELU) val[v] = fmaxf(val[v], 0.f);
      }
      const int co = mt * 16 + 4 * g;
      if (OUTF32) {
        *reinterpret_cast<f4*>(&out_f[(size_t)(y * HW + x) * COUT + co]) = f4{val[0], val[1], val[2], val[3]};
      } else {
        *reinterpret_cast<s4*>(&Xout[((y + 1) * HALO + x + 1) * COUT + co]) =
            s4{f2bf(val[0]), f2bf(val[1]), f2bf(val[2]), f2bf(val[3])};
      }
    }
  }
  __syncthreads();   // the output tile is complete and the weights are free
}

__global__ void __launch_bounds__(NT) forward_fused_kernel(const short* in, const short* wb,
                                                           const float* p32, int ow0, int ow1,
                                                           int ow2, int ow3, int ob0, int ob1,
                                                           int ob2, int ob3, float* out) {
  constexpr int KPMAX = kpad<32>();
  __shared__ __attribute__((aligned(16))) short X8[HALO * HALO * 8];
  __shared__ __attribute__((aligned(16))) short Xa[HALO * HALO * 32];
  __shared__ __attribute__((aligned(16))) short Xb[HALO * HALO * 32];
  __shared__ __attribute__((aligned(16))) short Ws[32 * KPMAX];
  const int b = blockIdx.x;
  // zero halos of the 32-channel tiles (their interiors are written whole
  // by every layer), then the input tile
  for (int e = threadIdx.x; e < HALO * HALO * 32 / 4; e += NT) {
    reinterpret_cast<s4*>(Xa)[e] = s4{0, 0, 0, 0};
    reinterpret_cast<s4*>(Xb)[e] = s4{0, 0, 0, 0};
  }
  load_halo<8>(in + (size_t)b * NPIX * 8, X8);
  conv_layer_lds<8, 32, true, false>(X8, wb + ow0, p32 + ob0, Ws, Xa, nullptr);
  conv_layer_lds<32, 32, true, false>(Xa, wb + ow1, p32 + ob1, Ws, Xb, nullptr);
  conv_layer_lds<32, 32, true, false>(Xb, wb + ow2, p32 + ob2, Ws, Xa, nullptr);
  conv_layer_lds<32, 16, false, true>(Xa, wb + ow3, p32 + ob3, Ws, nullptr, out + (size_t)b * NPIX * 16);
}

// ---------------------------------------------------------------------------
// backward to the input: dx[q][ci] = sum_{tap,co} W[co][tap][ci] gy[q - off(tap)][co],
// multiplied by the ReLU mask of the previous layer's output (y_prev > 0)
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ void __launch_bounds__(NT) conv_bwd_data_kernel(const short* gy, const short* W,
                                                           const short* yprev, short* gx) {
  constexpr int KP = kpad<CIN>();
  constexpr int K2 = 9 * COUT;       // (tap, co), a multiple of 16
  __shared__ __attribute__((aligned(16))) short Gs[HALO * HALO * COUT];
  __shared__ __attribute__((aligned(16))) short Wt[CIN * K2];
  const int b = blockIdx.x;
  for (int e = threadIdx.x; e < CIN * K2; e += NT) {
    const int ci = e / K2, r = e % K2, tap = r / COUT, co = r % COUT;
    Wt[e] = W[co * KP + tap * CIN + ci];
  }
  load_halo<COUT>(gy + (size_t)b * NPIX * COUT, Gs);
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int x = lane & 15, g = lane >> 4;
  for (int mt = 0; mt < CIN / 16 + (CIN % 16 ? 1 : 0); ++mt) {
    for (int yy = 0; yy < 4; ++yy) {
      const int y = wv * 4 + yy;
      f4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll 4
      for (int kk = 0; kk < K2 / 16; ++kk) {
        const int k0 = 16 * kk + 4 * g, tap = k0 / COUT, co = k0 % COUT;
        const int dy = tap / 3 - 1, dx = tap % 3 - 1;
        const s4 bv = *reinterpret_cast<const s4*>(&Gs[((y - dy + 1) * HALO + x - dx + 1) * COUT + co]);
        const int ci = mt * 16 + x;
        s4 av = {0, 0, 0, 0};
        if (ci < CIN) av = *reinterpret_cast<const s4*>(&Wt[ci * K2 + k0]);
        acc = mma(av, bv, acc);
      }
      const int p = y * HW + x;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int ci = mt * 16 + 4 * g + v;
        if (ci >= CIN) continue;
        const size_t o = ((size_t)b * NPIX + p) * CIN + ci;
        gx[o] = bf2f(yprev[o]) > 0.f ? f2bf(acc[v]) : (short)0;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// weight gradient: dW[co][tap][ci] = sum_{b,p} gy[b][p][co] x[b][p + off(tap)][ci],
// db[co] = sum gy; each work-group reduces a chunk of patches into its own
// slot of `part` (COUT*KP + COUT floats), summed later in a fixed order.
// ---------------------------------------------------------------------------
template <int CIN, int COUT>
__global__ void __launch_bounds__(NT) conv_bwd_weight_kernel(const short* gy, const short* xin,
                                                             float* part, int nbatch, int chunk) {
  constexpr int KP = kpad<CIN>();
  constexpr int MT = COUT / 16, NTL = KP / 16, TILES = MT * NTL;
  constexpr int PER_WAVE = (TILES + 3) / 4;
  __shared__ __attribute__((aligned(16))) short Gs[NPIX * COUT];
  __shared__ __attribute__((aligned(16))) short Xs[HALO * HALO * CIN];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int j = lane & 15, g = lane >> 4;
  f4 acc[PER_WAVE];
  for (int q = 0; q < PER_WAVE; ++q) acc[q] = f4{0.f, 0.f, 0.f, 0.f};
  float bsum = 0.f;
  const int b0 = blockIdx.x * chunk, b1 = min(nbatch, b0 + chunk);
  for (int b = b0; b < b1; ++b) {
    __syncthreads();
    for (int e = threadIdx.x; e < NPIX * COUT; e += NT) Gs[e] = gy[(size_t)b * NPIX * COUT + e];
    load_halo<CIN>(xin + (size_t)b * NPIX * CIN, Xs);
    __syncthreads();
    if (threadIdx.x < COUT)
      for (int p = 0; p < NPIX; ++p) bsum += bf2f(Gs[p * COUT + threadIdx.x]);
    for (int q = 0; q < PER_WAVE; ++q) {
      const int tile = wv * PER_WAVE + q;
      if (tile >= TILES) break;
      const int mt = tile / NTL, nt = tile % NTL;
      const int co = mt * 16 + j;                  // A row (this lane)
      const int n = nt * 16 + j;                   // B column (this lane)
      const int tap = n / CIN, ci = n % CIN;
      const int dy = tap / 3 - 1, dx = tap % 3 - 1;
      f4 a4 = acc[q];
      for (int kk = 0; kk < NPIX / 16; ++kk) {     // 16 pixels per step: image row kk
        s4 av, bv;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int xx = 4 * g + e;                // pixel (xx, kk)
          av[e] = Gs[(kk * HW + xx) * COUT + co];
          bv[e] = (tap < 9) ? Xs[((kk + dy + 1) * HALO + xx + dx + 1) * CIN + ci] : (short)0;
        }
        a4 = mma(av, bv, a4);
      }
      acc[q] = a4;
    }
  }
  float* out = part + (size_t)blockIdx.x * (COUT * KP + COUT);
  for (int q = 0; q < PER_WAVE; ++q) {
    const int tile = wv * PER_WAVE + q;
    if (tile >= TILES) break;
    const int mt = tile / NTL, nt = tile % NTL;
#pragma unroll
    for (int v = 0; v < 4; ++v) out[(mt * 16 + 4 * g + v) * KP + nt * 16 + j] = acc[q][v];
  }
  if (threadIdx.x < COUT) out[COUT * KP + threadIdx.x] = bsum;
}

// sum the per-chunk partial gradients in chunk order
__global__ void reduce_parts_kernel(const float* part, int nchunks, int len, float* grad) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < len; i += gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int c = 0; c < nchunks; ++c) s += part[(size_t)c * len + i];
    grad[i] = s;
  }
}

// mean squared error over all outputs; gradient into BF16 (channels-last)
__global__ void __launch_bounds__(NT) mse_kernel(const float* pred, const float* target, size_t n,
                                                 float scale, short* grad, float* part) {
  __shared__ float red[NT];
  float s = 0.f;
  for (size_t i = blockIdx.x * (size_t)NT + threadIdx.x; i < n; i += (size_t)gridDim.x * NT) {
    const float d = pred[i] - target[i];
    s += d * d;
    grad[i] = f2bf(2.f * d * scale);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = NT / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void adam_kernel(float* p, const float* grad, float* m, float* v, int n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gr = grad[i];
    const float mi = b1 * m[i] + (1.f - b1) * gr;
    const float vi = b2 * v[i] + (1.f - b2) * gr * gr;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

// FP32 master parameters -> BF16 weights of the four layers
__global__ void cast_weights_kernel(const float* p, short* wb, int n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    wb[i] = f2bf(p[i]);
}

}  // namespace cnn
}  // namespace mrcm

// ===========================================================================
// host side: parameter layout, network object, C ABI
// ===========================================================================

#include "../../include/mrcm.h"

#include <stdio.h>
#include <string.h>

#include <new>
#include <string>
#include <vector>

namespace mrcm {
namespace cnn {

const int CIN_P[NLAYERS] = {8, 32, 32, 32};
const int CIN_REAL[NLAYERS] = {5, 32, 32, 32};
const int COUT_L[NLAYERS] = {32, 32, 32, 16};

int kp_of(int l) { return (9 * CIN_P[l] + 15) / 16 * 16; }
int wlen(int l) { return COUT_L[l] * kp_of(l); }
int off_w(int l) {
  int o = 0;
  for (int q = 0; q < l; ++q) o += wlen(q) + COUT_L[q];
  return o;
}
int off_b(int l) { return off_w(l) + wlen(l); }
int n_params() { return off_w(NLAYERS); }

hipError_t forward(const short* in, const short* wb, const float* p32, short* a1, short* a2,
                   short* a3, float* out, int batch, hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL((conv_fwd_kernel<8, 32, true, false>), dim3(batch), dim3(NT), 0, st, in,
                     wb + off_w(0), p32 + off_b(0), a1, nullptr);
  hipLaunchKernelGGL((conv_fwd_kernel<32, 32, true, false>), dim3(batch), dim3(NT), 0, st, a1,
                     wb + off_w(1), p32 + off_b(1), a2, nullptr);
  hipLaunchKernelGGL((conv_fwd_kernel<32, 32, true, false>), dim3(batch), dim3(NT), 0, st, a2,
                     wb + off_w(2), p32 + off_b(2), a3, nullptr);
  hipLaunchKernelGGL((conv_fwd_kernel<32, 16, false, true>), dim3(batch), dim3(NT), 0, st, a3,
                     wb + off_w(3), p32 + off_b(3), nullptr, out);
  return hipGetLastError();
}

hipError_t forward_fused(const short* in, const short* wb, const float* p32, float* out, int batch,
                         hipStream_t st) {
  if (batch <= 0) return hipSuccess;
  hipLaunchKernelGGL(forward_fused_kernel, dim3(batch), dim3(NT), 0, st, in, wb, p32, off_w(0), off_w(1),
                     off_w(2), off_w(3), off_b(0), off_b(1), off_b(2), off_b(3), out);
  return hipGetLastError();
}

hipError_t cast(const float* p32, short* wb, hipStream_t st) {
  hipLaunchKernelGGL(cast_weights_kernel, dim3(64), dim3(256), 0, st, p32, wb, n_params());
  return hipGetLastError();
}

}  // namespace cnn
}  // namespace mrcm

using namespace mrcm;

struct mrcm_cnn {
  hipStream_t st = nullptr;
  bool own_stream = false;
  int max_batch = 0;
  int chunk = 8;
  long long step = 0;
  float *p32 = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
  short* wb = nullptr;
  short *a1 = nullptr, *a2 = nullptr, *a3 = nullptr;
  float* out = nullptr;
  short *g4 = nullptr, *g3 = nullptr, *g2 = nullptr, *g1 = nullptr;
  float* part = nullptr;
  float* loss_part = nullptr;
  std::vector<void*> allocs;
};

namespace {

constexpr int LOSS_WG = 256;

template <class T>
int cnn_alloc(mrcm_cnn* n, T** p, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, (count ? count : 1) * sizeof(T)) != hipSuccess) return MRCM_E_NOMEM;
  n->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return MRCM_OK;
}

#define CNN_ALLOC(n, p, c)                          \
  do {                                              \
    int r_ = cnn_alloc(n, &(p), (size_t)(c));       \
    if (r_ != MRCM_OK) return r_;                   \
  } while (0)
#define CNN_HIP(call)                               \
  do {                                              \
    if ((call) != hipSuccess) return MRCM_E_HIP;    \
  } while (0)

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

double gauss(uint64_t& s) {
  const double u1 = ((splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  const double u2 = ((splitmix(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

// He-normal initial weights; padded taps and channels stay zero
std::vector<float> initial_params(uint64_t seed) {
  using namespace mrcm::cnn;
  std::vector<float> p(n_params(), 0.f);
  uint64_t s = seed ^ 0x5DEECE66Dull;
  for (int l = 0; l < NLAYERS; ++l) {
    const double sd = sqrt(2.0 / (9.0 * CIN_REAL[l]));
    const int kp = kp_of(l);
    for (int co = 0; co < COUT_L[l]; ++co)
      for (int tap = 0; tap < 9; ++tap)
        for (int ci = 0; ci < CIN_REAL[l]; ++ci)
          p[off_w(l) + co * kp + tap * CIN_P[l] + ci] = (float)(sd * gauss(s));
  }
  return p;
}

// loss and gradient of one batch; leaves the gradient in net->grad and the
// loss partials in net->loss_part
int backprop(mrcm_cnn* net, const short* in, const float* target, int batch) {
  using namespace mrcm::cnn;
  hipStream_t st = net->st;
  CNN_HIP(forward(in, net->wb, net->p32, net->a1, net->a2, net->a3, net->out, batch, st));
  const size_t nout = (size_t)batch * NPIX * 16;
  hipLaunchKernelGGL(mse_kernel, dim3(LOSS_WG), dim3(NT), 0, st, net->out, target, nout,
                     1.0f / (float)nout, net->g4, net->loss_part);
  const int nch = (batch + net->chunk - 1) / net->chunk;
  // layer 4
  hipLaunchKernelGGL((conv_bwd_weight_kernel<32, 16>), dim3(nch), dim3(NT), 0, st, net->g4, net->a3,
                     net->part, batch, net->chunk);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(64), dim3(256), 0, st, net->part, nch,
                     wlen(3) + COUT_L[3], net->grad + off_w(3));
  hipLaunchKernelGGL((conv_bwd_data_kernel<32, 16>), dim3(batch), dim3(NT), 0, st, net->g4,
                     net->wb + off_w(3), net->a3, net->g3);
  // layer 3
  hipLaunchKernelGGL((conv_bwd_weight_kernel<32, 32>), dim3(nch), dim3(NT), 0, st, net->g3, net->a2,
                     net->part, batch, net->chunk);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(64), dim3(256), 0, st, net->part, nch,
                     wlen(2) + COUT_L[2], net->grad + off_w(2));
  hipLaunchKernelGGL((conv_bwd_data_kernel<32, 32>), dim3(batch), dim3(NT), 0, st, net->g3,
                     net->wb + off_w(2), net->a2, net->g2);
  // layer 2
  hipLaunchKernelGGL((conv_bwd_weight_kernel<32, 32>), dim3(nch), dim3(NT), 0, st, net->g2, net->a1,
                     net->part, batch, net->chunk);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(64), dim3(256), 0, st, net->part, nch,
                     wlen(1) + COUT_L[1], net->grad + off_w(1));
  hipLaunchKernelGGL((conv_bwd_data_kernel<32, 32>), dim3(batch), dim3(NT), 0, st, net->g2,
                     net->wb + off_w(1), net->a1, net->g1);
  // layer 1 (no gradient with respect to the network input)
  hipLaunchKernelGGL((conv_bwd_weight_kernel<8, 32>), dim3(nch), dim3(NT), 0, st, net->g1, in,
                     net->part, batch, net->chunk);
  hipLaunchKernelGGL(reduce_parts_kernel, dim3(64), dim3(256), 0, st, net->part, nch,
                     wlen(0) + COUT_L[0], net->grad + off_w(0));
  CNN_HIP(hipGetLastError());
  return MRCM_OK;
}

int read_loss(mrcm_cnn* net, float* loss, int batch) {
  std::vector<float> lp(LOSS_WG);
  CNN_HIP(hipMemcpyAsync(lp.data(), net->loss_part, LOSS_WG * sizeof(float), hipMemcpyDeviceToHost,
                         net->st));
  CNN_HIP(hipStreamSynchronize(net->st));
  double s = 0.0;
  for (float v : lp) s += v;
  if (loss) *loss = (float)(s / ((double)batch * mrcm::cnn::NPIX * 16));
  return MRCM_OK;
}

}  // namespace

extern "C" {

int mrcm_cnn_create(mrcm_cnn** out, int32_t max_batch, uint64_t seed, void* hip_stream) {
  using namespace mrcm::cnn;
  if (!out || max_batch <= 0) return MRCM_E_INVAL;
  *out = nullptr;
  mrcm_cnn* net = new (std::nothrow) mrcm_cnn();
  if (!net) return MRCM_E_NOMEM;
  auto body = [&]() -> int {
    net->max_batch = max_batch;
    if (hip_stream) {
      net->st = (hipStream_t)hip_stream;
    } else {
      CNN_HIP(hipStreamCreate(&net->st));
      net->own_stream = true;
    }
    const int np = n_params();
    CNN_ALLOC(net, net->p32, np);
    CNN_ALLOC(net, net->grad, np);
    CNN_ALLOC(net, net->m, np);
    CNN_ALLOC(net, net->v, np);
    CNN_ALLOC(net, net->wb, np);
    const size_t B = (size_t)max_batch;
    CNN_ALLOC(net, net->a1, B * NPIX * 32);
    CNN_ALLOC(net, net->a2, B * NPIX * 32);
    CNN_ALLOC(net, net->a3, B * NPIX * 32);
    CNN_ALLOC(net, net->out, B * NPIX * 16);
    CNN_ALLOC(net, net->g4, B * NPIX * 16);
    CNN_ALLOC(net, net->g3, B * NPIX * 32);
    CNN_ALLOC(net, net->g2, B * NPIX * 32);
    CNN_ALLOC(net, net->g1, B * NPIX * 32);
    int maxlen = 0;
    for (int l = 0; l < NLAYERS; ++l) maxlen = std::max(maxlen, wlen(l) + COUT_L[l]);
    CNN_ALLOC(net, net->part, ((B + net->chunk - 1) / net->chunk) * (size_t)maxlen);
    CNN_ALLOC(net, net->loss_part, LOSS_WG);
    std::vector<float> p = initial_params(seed);
    std::vector<float> z(np, 0.f);
    CNN_HIP(hipMemcpy(net->p32, p.data(), np * sizeof(float), hipMemcpyHostToDevice));
    CNN_HIP(hipMemcpy(net->m, z.data(), np * sizeof(float), hipMemcpyHostToDevice));
    CNN_HIP(hipMemcpy(net->v, z.data(), np * sizeof(float), hipMemcpyHostToDevice));
    CNN_HIP(cast(net->p32, net->wb, net->st));
    CNN_HIP(hipStreamSynchronize(net->st));
    return MRCM_OK;
  };
  const int rc = body();
  if (rc != MRCM_OK) {
    mrcm_cnn_destroy(net);
    return rc;
  }
  *out = net;
  return MRCM_OK;
}

int mrcm_cnn_num_params(const mrcm_cnn* net, int32_t* n) {
  if (!net || !n) return MRCM_E_INVAL;
  *n = mrcm::cnn::n_params();
  return MRCM_OK;
}

int mrcm_cnn_get_params(mrcm_cnn* net, float* params) {
  if (!net || !params) return MRCM_E_INVAL;
  CNN_HIP(hipMemcpyAsync(params, net->p32, mrcm::cnn::n_params() * sizeof(float),
                         hipMemcpyDeviceToHost, net->st));
  CNN_HIP(hipStreamSynchronize(net->st));
  return MRCM_OK;
}

int mrcm_cnn_set_params(mrcm_cnn* net, const float* params) {
  if (!net || !params) return MRCM_E_INVAL;
  CNN_HIP(hipMemcpyAsync(net->p32, params, mrcm::cnn::n_params() * sizeof(float),
                         hipMemcpyHostToDevice, net->st));
  CNN_HIP(mrcm::cnn::cast(net->p32, net->wb, net->st));
  CNN_HIP(hipStreamSynchronize(net->st));
  return MRCM_OK;
}

int mrcm_cnn_forward(mrcm_cnn* net, const void* inputs, float* outputs, int32_t batch) {
  if (!net || !inputs || !outputs || batch <= 0 || batch > net->max_batch) return MRCM_E_INVAL;
  CNN_HIP(mrcm::cnn::forward_fused((const short*)inputs, net->wb, net->p32, outputs, batch, net->st));
  CNN_HIP(hipStreamSynchronize(net->st));
  return MRCM_OK;
}

int mrcm_cnn_loss_grad(mrcm_cnn* net, const void* inputs, const float* targets, int32_t batch,
                       float* loss, float* grads) {
  if (!net || !inputs || !targets || batch <= 0 || batch > net->max_batch) return MRCM_E_INVAL;
  int rc = backprop(net, (const short*)inputs, targets, batch);
  if (rc != MRCM_OK) return rc;
  if (grads)
    CNN_HIP(hipMemcpyAsync(grads, net->grad, mrcm::cnn::n_params() * sizeof(float),
                           hipMemcpyDeviceToHost, net->st));
  return read_loss(net, loss, batch);
}

int mrcm_cnn_train_step(mrcm_cnn* net, const void* inputs, const float* targets, int32_t batch,
                        float lr, float* loss) {
  if (!net || !inputs || !targets || batch <= 0 || batch > net->max_batch || !(lr > 0.f))
    return MRCM_E_INVAL;
  int rc = backprop(net, (const short*)inputs, targets, batch);
  if (rc != MRCM_OK) return rc;
  net->step += 1;
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.f - powf(b1, (float)net->step), c2 = 1.f - powf(b2, (float)net->step);
  hipLaunchKernelGGL(mrcm::cnn::adam_kernel, dim3(64), dim3(256), 0, net->st, net->p32, net->grad,
                     net->m, net->v, mrcm::cnn::n_params(), lr, b1, b2, 1e-8f, c1, c2);
  CNN_HIP(hipGetLastError());
  CNN_HIP(mrcm::cnn::cast(net->p32, net->wb, net->st));
  if (loss) return read_loss(net, loss, batch);
  CNN_HIP(hipStreamSynchronize(net->st));
  return MRCM_OK;
}

void mrcm_cnn_destroy(mrcm_cnn* net) {
  if (!net) return;
  if (net->st) (void)hipStreamSynchronize(net->st);
  for (void* q : net->allocs) (void)hipFree(q);
  if (net->own_stream && net->st) (void)hipStreamDestroy(net->st);
  delete net;
}

}  // extern "C"

// access for the solver context (api.hip)
namespace mrcm {
namespace cnn {
const float* params_of(const mrcm_cnn* net) { return net->p32; }
hipStream_t stream_of(const mrcm_cnn* net) { return net->st; }
}  // namespace cnn
}  // namespace mrcm
