// Internal declarations of the MRCM library: device argument blocks, tree
// node descriptors and kernel launchers.  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mrcm {

// status bits raised by kernels (device int, read back after a solve)
enum : int {
  ST_BAD_LAMBDA = 1,    // a mobility was not finite and positive
  ST_LOCAL_PIVOT = 2,   // a Gauss-Jordan pivot of a local Schur block was not positive
  ST_IFACE_PIVOT = 4,   // a pivot of the interface elimination was zero or not finite
  ST_STITCH_PIVOT = 8,  // a pivot of the stitch re-solve was not positive
};

// Problem geometry shared by the per-subdomain kernels.
struct Geo {
  int nx, ny;       // cells
  int M;            // subdomain edge in cells (square subdomains)
  int SX, SY;       // subdomains per direction
  int nV;           // number of vertical interfaces
  int n_sub;
  int nP, nU, D;    // interface dofs per interface (D = nP + nU)
  int kind[4];      // boundary kind per side W E S N (1 = Dirichlet)
  int gauge;        // 1: no Dirichlet side, first pressure dof pinned
  int generic;      // 1: use the generic per-subdomain kernels even where a
                    //    specialised one exists (host-side switch)
  int prec;         // 0: FP64 local solves, 1: FP32 + FP64 iterative refinement,
                    // 2: surrogate + residual gate + FP64 re-solve
  double hx, hy;
  double tfx, tfy;  // half-cell transmissibility per unit kappa: hy / (hx / 2), hx / (hy / 2)
  double grav;      // gravity along y, g dh/dy (used where SubArgs::rho is set)
};

// Device data of a context used by the subdomain kernels.
struct SubArgs {
  Geo g;
  const double* K;        // nx*ny absolute permeability
  const double* lam;      // nx*ny total mobility
  const double* src;      // nx*ny source per unit area, or nullptr
  const double* rho;      // nx*ny lambda_g / lambda (gravity), or nullptr (no gravity)
  const int2* nact;       // per interface: active pressure / flux functions (physics
                          // spaces; the other slots are zero), or nullptr (all active)
  const double* bcv[4];   // boundary values per side (ny, ny, nx, nx)
  const double* alpha;    // per interface
  const double* basis;    // [iface][D][M]: rows 0..nP-1 pressure, nP..D-1 flux functions
  double* X;              // [sub][R][M*M] local solutions (R = 1 + 4D), column-major per subdomain
  double* blocks;         // [sub][4D][4D+1] symmetric local interface blocks
  const double* coef;     // interface solution (stitch kernel)
  double* p_out;          // nx*ny composed pressure (stitch kernel)
  double* ux;             // (nx+1)*ny
  double* uy;             // nx*(ny+1)
  double* sub_stats;      // [sub][3]: max cell imbalance, max |F|, sum of p
  int* status;
  int* fallback;          // FP32 refinement: [0] = count, [1..] = subdomains to redo in FP64
  int* ir_iters;          // FP32 refinement: [0] = largest refinement count used
  double gate_tol;        // surrogate: accepted if ||b - A x|| <= gate_tol ||b|| per column
  int ir_max;             // FP32 refinement: at most this many steps
  double ir_tol;          // FP32 refinement: converged (and accepted without the FP64
                          // re-solve) once the last correction is <= ir_tol of the solution
  double* scratch;        // generic kernels: per-subdomain work arrays (global memory)
  long long scratch_stride;   // doubles per subdomain in scratch
  unsigned long long* stamps; // phase clock readings (PhaseStamp slots)
};

// Phase boundaries, read from the GPU's constant-rate clock by the kernels
// that open or close a phase (thread 0 of work-group 0 at its start, or the
// single work-group of a reduction at its end), so that timing the phases
// adds no packet to the stream.
enum PhaseStamp {
  STAMP_SOLVE = 0,       // solve enqueued: the local kernels follow
  STAMP_IFACE = 1,       // first interface kernel starts
  STAMP_IFACE_END = 2,   // interface residual reduced (after any refinement)
  STAMP_FLUX = 3,        // stitch starts
  STAMP_FLUX_END = 4,    // flux statistics reduced
  STAMP_N = 5
};
__device__ inline void stamp_now(unsigned long long* s) { *s = __builtin_amdgcn_s_memrealtime(); }

// Frontal-matrix node of the nested-dissection elimination of the
// interface system.  Front F is n x (n+1), row-major, last column = rhs;
// the first s unknowns are eliminated at this node.
struct NodeDesc {
  long long f_off;      // offset of F in the tree buffer (doubles)
  long long map_off;    // offset into the map array (n int2: child A index, child B index)
  long long dof_off;    // offset into the dof array (n ints: global dof per position)
  long long c_off[2];   // offset of each child's Schur block (top-left)
  long long inv_off;    // blocked fronts: offset of the per-panel diagonal-block inverses
  int n, s;
  int c_ld[2];          // row stride of each child's Schur block
  int c_rhs[2];         // rhs column of each child's Schur block (relative to c_off)
  int blocked;          // 0: eliminated pivot by pivot (classic in-place LU);
                        // 1: eliminated by panels of PANEL_NB columns
  long long r_off;      // offset of the front's right-hand-side vector (n) in the rhs tree
  long long cr_off[2];  // each child's right-hand-side vector, -1 for a leaf child
};

struct PanelItem {      // one work-group of a blocked trailing update
  int node;             // index into the node descriptor array
  int i0, j0;           // first row / column of the 64 x 64 tile
  int pad;              // 0: tile; 1: tile whose leading 32 x 32 block is the next
                        // panel's diagonal block (left out); 2: that block alone,
                        // updated and inverted (i0 = j0 = its first row);
                        // 3 (first panel of a front without trailing rows):
                        // the panel's rows from column j0, stored as assembled
  int n, s;             // the front's size and separator size (copied from its node)
  long long f_off;      // the front's offset in the tree buffer
  long long inv_off;    // the front's diagonal-block inverses
};

// ---- launchers (local.hip) ----
hipError_t launch_local_basis(const SubArgs& a, hipStream_t st);
hipError_t launch_stitch(const SubArgs& a, hipStream_t st);
hipError_t launch_mobility(const double* in, double* lam, size_t n, int from_saturation,
                           double mu_w, double mu_o, hipStream_t st);
// total mobility and lambda_g / lambda from a saturation (gravity)
hipError_t launch_mobility_gravity(const double* s, double* lam, double* rho, size_t n, double mu_w,
                                   double mu_o, double rho_w, double rho_o, hipStream_t st);
hipError_t launch_finish_flux(const SubArgs& a, double* result, hipStream_t st);
// (local_mfma.hip) 16 x 16 subdomains, 2 + 2 interface dofs (FP64: two wavefronts per subdomain)
hipError_t launch_basis_m16d4(const SubArgs& a, hipStream_t st);
// FP32 factors and solves with FP64 iterative refinement; subdomains that do
// not converge are listed in a.fallback and re-solved by the FP64 kernel
hipError_t launch_basis32_m16d4(const SubArgs& a, hipStream_t st);
hipError_t launch_basis_m16d4_list(const SubArgs& a, hipStream_t st);
hipError_t launch_stitch_m16d4(const SubArgs& a, hipStream_t st);
// 16 x 16 subdomains with 8 dofs per side (physics-based spaces, 4 + 4 slots):
// two work-groups per subdomain, one per window of 4 dofs per side
hipError_t launch_basis_m16d8(const SubArgs& a, hipStream_t st);
hipError_t launch_stitch_m16d8(const SubArgs& a, hipStream_t st);
// (local_mfma32.hip) 32 x 32 subdomains, 4 dofs per side (2 + 2) or 8 (FP64
// only, two windows of 4): FP64 basis functions on the matrix cores; list =
// only the FP32 fallback list
bool basis32x32_supported(const Geo& g);
long long basis32x32_scratch(const Geo& g);   // doubles of per-subdomain scratch they need
hipError_t launch_basis32x32(const SubArgs& a, hipStream_t st, bool list);
hipError_t launch_stitch32x32(const SubArgs& a, hipStream_t st);
bool local_supported(int M, int D);
// sizes with an FP32 + refinement kernel (16 x 16 with 2 + 2 dofs, 32 x 32 with 4 dofs)
bool local_fp32_supported(int M, int D, int nP);
// doubles of global scratch per subdomain the generic kernels need (0 if none)
long long local_scratch_doubles(const Geo& g);

// ---- launchers (interface.hip) ----
// stamp: if not NULL, the launch's start is written there
hipError_t launch_front_small(const NodeDesc* nodes, int count, int max_n, double* tree,
                              const int2* maps, int* status, unsigned long long* stamp,
                              hipStream_t st);
// one panel of the blocked fronts of a level; the first (k0 = 0) also
// assembles the fronts from their children
hipError_t launch_front_update(const NodeDesc* nodes, const PanelItem* items, int count, int k0,
                               double* tree, const int2* maps, double* inv, int* status,
                               unsigned long long* stamp, hipStream_t st);
// back substitution of one tree level; rtree = NULL takes the right-hand
// side from the fronts' last column, else from the fronts' rhs vectors
hipError_t launch_front_back(const NodeDesc* nodes, int count, int max_n, const double* tree,
                             const double* inv, const int* dofs, const double* rtree, double* x,
                             hipStream_t st);
// forward elimination of a new right-hand side r (one value per interface
// dof) through the stored fronts of one tree level, into the rhs tree
hipError_t launch_front_rhs(const NodeDesc* nodes, int count, int max_n, const double* tree,
                            const double* inv, const int2* maps, const int* dofs, const double* r,
                            double* rtree, hipStream_t st);
// r = b - A x of the assembled interface system (double-double), written to
// r if not NULL; partials: 2 doubles per work-group (RESID_WG of them),
// reduced into out2[0] = max|r|, out2[1] = max|b|; the reduction's end is
// written to stamp
hipError_t launch_iface_residual(const Geo& g, const double* blocks, const double* x, double* r,
                                 double* partials, double* out2, unsigned long long* stamp,
                                 hipStream_t st);
// x += dx over n values
hipError_t launch_add(double* x, const double* dx, int n, hipStream_t st);
constexpr int RESID_WG = 128;

hipError_t launch_copy(double* dst, const double* src, size_t n, hipStream_t st);

// ---- surrogate network (surrogate.hip) ----
}  // namespace mrcm
struct mrcm_cnn;
namespace mrcm {
namespace cnn {
int n_params();
int off_w(int l);
int off_b(int l);
// forward pass of the network: in BF16 [batch][256][8] -> out FP32 [batch][256][16]
hipError_t forward(const short* in, const short* wb, const float* p32, short* a1, short* a2,
                   short* a3, float* out, int batch, hipStream_t st);
// the same outputs from one launch that keeps the activations on chip
// (inference only: the per-layer form keeps them for the backward pass)
hipError_t forward_fused(const short* in, const short* wb, const float* p32, float* out, int batch,
                         hipStream_t st);
hipError_t cast(const float* p32, short* wb, hipStream_t st);
const float* params_of(const mrcm_cnn* net);
hipStream_t stream_of(const mrcm_cnn* net);
}  // namespace cnn
// (local_mfma.hip) surrogate inputs / training targets / residual gate for
// 16 x 16 subdomains with 2 + 2 dofs
hipError_t launch_surrogate_inputs(const SubArgs& a, short* inputs, hipStream_t st);
hipError_t launch_surrogate_targets(const SubArgs& a, float* targets, hipStream_t st);
hipError_t launch_surrogate_gate(const SubArgs& a, const float* pred, hipStream_t st);

constexpr int PANEL_NB = 32;      // panel width of the blocked elimination
constexpr int TILE = 64;          // trailing-update tile
constexpr int SMALL_FRONT = 64;   // levels with fronts up to this size are eliminated in registers
constexpr int MAX_FRONT = 4096;   // largest front the interface plan accepts

}  // namespace mrcm
