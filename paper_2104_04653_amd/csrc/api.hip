// C ABI of the MRCM library: context, validation, set-up of the interface
// spaces and of the nested-dissection plan for the interface system, and
// the orchestration of the per-step kernels.  Declarations and the contract
// of every entry point are in include/mrcm.h.
#include "../../include/mrcm.h"
#include "mrcm_internal.h"
#include "physics_space.h"
#include "transport.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <mutex>
#include <new>
#include <string>
#include <unordered_map>
#include <vector>

using namespace mrcm;
using namespace mrcm::phys;

// Scratch of mrcm_fine_flux_static: the stitch's per-subdomain statistics
// (max cell imbalance, max |F|, pressure sum: 3 doubles per subdomain) and
// the two values they reduce to, in a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends) instead of
// context memory.  Host code never passes the array's name to a kernel: its
// device address is taken once per device with hipGetSymbolAddress.
constexpr int STATIC_MAX_SUB = 65536;
constexpr size_t STATIC_SCRATCH_DOUBLES = 3 * (size_t)STATIC_MAX_SUB + 2;
static __device__ __align__(256) double scratch[STATIC_SCRATCH_DOUBLES];

namespace {

struct PanelLaunch {
  int k0;
  int diag_off, diag_count;     // fronts with a panel at k0 (into the id array)
  int update_off, update_count; // trailing tiles (into the item array)
};

struct LevelPlan {
  bool small;
  int max_n, max_s;
  int ids_off, count;
  std::vector<PanelLaunch> panels;
};

}  // namespace

struct mrcm_ctx {
  std::string err;
  Geo g{};
  int precision = 0;
  int space = 0;
  double mu_w = 1.0, mu_o = 1.0;
  hipStream_t st = nullptr;
  bool own_stream = false;
  int n_dof = 0;
  int R = 0;
  bool solved = false;
  mrcm_stats stats{};

  // device buffers
  double *K = nullptr, *lam = nullptr, *stage = nullptr, *src = nullptr;
  double* bcv[4] = {nullptr, nullptr, nullptr, nullptr};
  double *alpha = nullptr, *basis = nullptr, *X = nullptr, *coef = nullptr;
  double *p = nullptr, *ux = nullptr, *uy = nullptr, *sub_stats = nullptr, *result = nullptr;
  double* tree = nullptr;
  // report block (one device allocation, read back with one copy):
  // result[RESULT_N] doubles, status, ir_iters, then the fallback list
  double* report = nullptr;
  int* status = nullptr;
  int* fallback = nullptr;     // FP32 refinement: count + list of subdomains
  int* ir_iters = nullptr;
  double* h_report = nullptr;  // pinned host mirror of the report head
  NodeDesc* d_nodes = nullptr;
  int2* d_maps = nullptr;
  int* d_dofs = nullptr;
  int* d_ids = nullptr;
  NodeDesc* d_lvnodes = nullptr;  // node descriptors in level order (ids order)
  PanelItem* d_items = nullptr;
  double* inv = nullptr;        // per-panel diagonal-block inverses of blocked fronts
  double* partials = nullptr;   // residual partial maxima
  double* rtree = nullptr;      // interface refinement: rhs vectors of the fronts
  double* rvec = nullptr;       // interface refinement: residual (n_dof)
  double* dx = nullptr;         // interface refinement: correction (n_dof)
  int iface_ir = 0;             // refinement steps taken by the last solve
  bool step_refined = false;    // the last mrcm_step refined its interface solve
  double* scratch = nullptr;    // generic local kernels: per-subdomain work arrays
  long long scratch_stride = 0;
  // surrogate precision: network parameters and per-subdomain activations
  float* s_p32 = nullptr;
  short* s_wb = nullptr;
  short* s_in = nullptr;
  float* s_pred = nullptr;
  bool s_ready = false;
  double gate_tol = 1e-6;
  // stopping rules of the iterative refinements (mrcm_set_refinement,
  // mrcm_set_interface_refinement); defaults set by mrcm_setup
  int ir_max = 0;
  double ir_tol = 0.0;
  int iface_ir_max = 0;
  double iface_ir_tol = 0.0;
  double iface_fail_tol = 0.0;
  std::vector<void*> allocs;

  // interface plan
  std::vector<LevelPlan> levels;
  long long leaf_block = 0;  // doubles per subdomain block
  double iface_flop = 0.0;   // algorithmic FLOP of one interface solve
  int iface_launches = 0;    // its kernel launches
  double* static_scratch = nullptr;       // this device's address of `scratch`
  // implicit transport: work arrays (set up with the context) and the
  // pinned mirror of its scalar block
  TransportArgs tr{};
  double* h_tscal = nullptr;
  double* s_prev = nullptr;               // SFI: the previous outer iterate
  // gravity variant: g dh/dy, phase densities, lambda_g / lambda per cell
  double grav = 0.0, rho_w = 0.0, rho_o = 0.0;
  double* rho = nullptr;
  bool rho_valid = false;                 // rho holds the last saturation's values
  // per interface: crossed by a high-permeability channel (adaptive alpha);
  // physics spaces: numbers of active pressure and flux functions
  std::vector<char> has_channel;
  int2* nact = nullptr;
  std::vector<int2> h_nact;               // host copy (the interface plan leaves inactive slots out)
  hipEvent_t ev[3] = {nullptr, nullptr, nullptr};   // solve start, local end, gate end
  unsigned long long* stamps = nullptr;   // device, inside the report block
  double clock_khz = 0.0;                 // rate of the clock the kernels read
};

namespace {

int fail(mrcm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(ctx, MRCM_E_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
int dev_alloc(mrcm_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  if (count == 0) count = 1;
  hipError_t e = hipMalloc(&q, count * sizeof(T));
  if (e != hipSuccess) return fail(c, MRCM_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
  c->allocs.push_back(q);
  *p = static_cast<T*>(q);
  return MRCM_OK;
}

#define ALLOC(ctx, ptr, n)                          \
  do {                                              \
    int r_ = dev_alloc(ctx, &(ptr), (size_t)(n));   \
    if (r_ != MRCM_OK) return r_;                   \
  } while (0)

bool finite_pos(double v) { return isfinite(v) && v > 0.0; }

// device address of `scratch`, looked up once per device (with that device
// current) and kept for the process
constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double* g_scratch_ptr[MAX_DEVICES] = {};

int bind_static_scratch(mrcm_ctx* c) {
  int dev = 0;
  HIPCHK(c, hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(c, MRCM_E_UNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(c, MRCM_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  c->static_scratch = g_scratch_ptr[dev];
  return MRCM_OK;
}

// report block: doubles result[0] = max cell imbalance, [1] = pressure sum
// (gauge shift), [2] = max |r|, [3] = max |b| of the interface residual,
// [STAMP_OFF + k] = clock reading of phase boundary k (PhaseStamp), as an
// unsigned 64-bit integer; then ints status, ir_iters, fallback count,
// fallback list
constexpr int STAMP_OFF = 4;
constexpr int RESULT_N = STAMP_OFF + STAMP_N + 1;
constexpr size_t REPORT_HEAD = RESULT_N * sizeof(double) + 3 * sizeof(int);

constexpr int IFACE_IR_MAX = 3;         // default refinement steps of the interface solve
// default max|r| / max|b| of the interface system that needs no refinement:
// near the FP64 floor for FP64 local solves; for FP32 + refinement, whose
// local solutions are converged to about 1e-10 relative, a residual 1e-12 of
// the right-hand side is already below what its inputs resolve
constexpr double IFACE_IR_TOL_FP64 = 1e-14;
constexpr double IFACE_IR_TOL_FP32 = 1e-12;
// default max|r| / max|b| above which a refined interface solve fails: the
// residual of an FP64 solution is about eps |A| |x|, which exceeds 1e-14
// of the right-hand side on ill-conditioned systems (all-Neumann wells at
// 256 x 256: 2.5e-13 after three steps, still within the 1e-10 parity of
// pressure and flux), so failure is declared only where digits that matter
// are lost
constexpr double IFACE_FAIL_TOL = 1e-10;
// default stopping rule of the FP32 local refinement: the last correction
// below 1e-12 of the solution, at most 8 steps.  The form's parity target
// against FP64 (1e-8) would be met at 1e-9, but the stitch's Neumann data
// are compatible only to the accuracy of the local solutions, and the cell
// balances of the stitched flux (1e-12 of the largest face flux) need local
// solutions near FP64 accuracy: refinement restores it
// BiCGSTAB of the transport's Newton steps: relative residual of the
// Jacobi-scaled system, iteration cap
constexpr double TRANSPORT_LIN_TOL = 1e-12;
constexpr int TRANSPORT_LIN_MAX = 400;
constexpr int LOCAL_IR_MAX = 8;
constexpr double LOCAL_IR_TOL = 1e-12;

// ---------------------------------------------------------------------------
// interface spaces, tabulated per interface on its fine faces
// ---------------------------------------------------------------------------

double hmean(double a, double b) { return 2.0 * a * b / (a + b); }

// Edge-solution functions on one interface: t_j = harmonic mean of K across
// face j; psi solves the 1-D two-point problem along the edge (conductance
// hmean(t_j, t_{j+1}) between neighbours, 2 t at the two ends) with psi = 1
// at the first end and 0 at the other.  Pressure functions {psi, 1 - psi},
// flux functions {t / mean t, t (psi - mean psi) / mean t}.  The conductances
// are in series, so psi at face j is the share of the total resistance
// between face j and the far end, and 1 - psi the share on the near side;
// both are formed as such sums, which keeps each accurate where it is small.
void edge_solution(const std::vector<double>& klo, const std::vector<double>& khi, double* out,
                   int M) {
  std::vector<double> t(M), near(M), far(M);
  for (int j = 0; j < M; ++j) t[j] = hmean(klo[j], khi[j]);
  const double r_first = 1.0 / (2.0 * t[0]), r_last = 1.0 / (2.0 * t[M - 1]);
  near[0] = r_first;
  for (int j = 1; j < M; ++j) near[j] = near[j - 1] + 1.0 / hmean(t[j - 1], t[j]);
  far[M - 1] = r_last;
  for (int j = M - 2; j >= 0; --j) far[j] = far[j + 1] + 1.0 / hmean(t[j], t[j + 1]);
  const double total = near[M - 1] + r_last;
  double tm = 0.0, pm = 0.0;
  for (int j = 0; j < M; ++j) {
    tm += t[j];
    pm += far[j] / total;
  }
  tm /= M;
  pm /= M;
  for (int j = 0; j < M; ++j) {
    const double psi = far[j] / total;
    out[0 * M + j] = psi;
    out[1 * M + j] = near[j] / total;
    out[2 * M + j] = t[j] / tm;
    out[3 * M + j] = t[j] * (psi - pm) / tm;
  }
}

// ---------------------------------------------------------------------------
// nested-dissection plan of the interface system
// ---------------------------------------------------------------------------

struct HNode {
  bool leaf = false;
  int sd = -1;
  int child[2] = {-1, -1};
  std::vector<int> dofs;   // frontal ordering: shared (eliminated) first
  int s = 0;
  int level = 0;
  long long f_off = 0;
};

struct TreeBuilder {
  int SX, SY, nV, D;
  std::vector<HNode> nodes;
  // physics spaces: slots of inactive functions (nP = pressure slots) are
  // not unknowns of the elimination: their coefficient is 0, their row and
  // column of the interface system are empty apart from a unit diagonal
  const std::vector<int2>* nact = nullptr;
  int nP = 0;
  int viface(int I, int J) const { return J * (SX - 1) + I; }
  int hiface(int I, int J) const { return nV + J * SX + I; }
  bool active(int e, int k) const {
    if (!nact) return true;
    const int2 n = (*nact)[e];
    return k < nP ? k < n.x : k - nP < n.y;
  }
  void add_dofs(std::vector<int>& out, int e) const {
    for (int k = 0; k < D; ++k)
      if (active(e, k)) out.push_back(e * D + k);
  }
  int rec(int I0, int I1, int J0, int J1) {
    if ((I1 - I0) * (J1 - J0) == 1) {
      HNode n;
      n.leaf = true;
      n.sd = J0 * SX + I0;
      nodes.push_back(n);
      return (int)nodes.size() - 1;
    }
    int a, b;
    std::vector<int> shared;
    if (I1 - I0 >= J1 - J0) {
      const int Im = (I0 + I1) / 2;
      a = rec(I0, Im, J0, J1);
      b = rec(Im, I1, J0, J1);
      for (int J = J0; J < J1; ++J) add_dofs(shared, viface(Im - 1, J));
    } else {
      const int Jm = (J0 + J1) / 2;
      a = rec(I0, I1, J0, Jm);
      b = rec(I0, I1, Jm, J1);
      for (int I = I0; I < I1; ++I) add_dofs(shared, hiface(I, Jm - 1));
    }
    HNode n;
    n.child[0] = a;
    n.child[1] = b;
    n.dofs = shared;
    n.s = (int)shared.size();
    if (I0 > 0) for (int J = J0; J < J1; ++J) add_dofs(n.dofs, viface(I0 - 1, J));
    if (I1 < SX) for (int J = J0; J < J1; ++J) add_dofs(n.dofs, viface(I1 - 1, J));
    if (J0 > 0) for (int I = I0; I < I1; ++I) add_dofs(n.dofs, hiface(I, J0 - 1));
    if (J1 < SY) for (int I = I0; I < I1; ++I) add_dofs(n.dofs, hiface(I, J1 - 1));
    n.level = 1 + std::max(nodes[a].level, nodes[b].level);
    nodes.push_back(n);
    return (int)nodes.size() - 1;
  }
  // position of global dof in the Schur block a child hands to its parent
  int schur_index(int node, int dof, const std::vector<std::unordered_map<int, int>>& pos) const {
    const HNode& n = nodes[node];
    if (n.leaf) {
      const int I = n.sd % SX, J = n.sd / SX;
      const int e = dof / D, k = dof % D;
      int side = -1;
      if (I > 0 && e == viface(I - 1, J)) side = 0;
      else if (I < SX - 1 && e == viface(I, J)) side = 1;
      else if (J > 0 && e == hiface(I, J - 1)) side = 2;
      else if (J < SY - 1 && e == hiface(I, J)) side = 3;
      return side < 0 ? -1 : side * D + k;
    }
    auto it = pos[node].find(dof);
    if (it == pos[node].end() || it->second < n.s) return -1;
    return it->second - n.s;
  }
};

int build_plan(mrcm_ctx* c) {
  const Geo& g = c->g;
  c->leaf_block = (long long)(4 * g.D) * (4 * g.D + 1);
  long long total = c->leaf_block * g.n_sub;
  if (c->n_dof == 0) {
    ALLOC(c, c->tree, total);
    return MRCM_OK;
  }
  TreeBuilder tb{g.SX, g.SY, g.nV, g.D, {}};
  if (!c->h_nact.empty()) {
    tb.nact = &c->h_nact;
    tb.nP = g.nP;
  }
  tb.nodes.reserve(2 * g.n_sub);
  const int root = tb.rec(0, g.SX, 0, g.SY);
  (void)root;
  std::vector<std::unordered_map<int, int>> pos(tb.nodes.size());
  for (size_t i = 0; i < tb.nodes.size(); ++i) {
    HNode& n = tb.nodes[i];
    if (n.leaf) continue;
    for (size_t k = 0; k < n.dofs.size(); ++k) pos[i][n.dofs[k]] = (int)k;
    n.f_off = total;
    total += (long long)n.dofs.size() * (n.dofs.size() + 1);
  }
  // descriptors, maps, dofs; non-leaf nodes grouped by level
  int max_level = 0;
  for (auto& n : tb.nodes) max_level = std::max(max_level, n.level);
  std::vector<NodeDesc> desc;
  std::vector<int2> maps;
  std::vector<int> dofs, ids;
  std::vector<PanelItem> items;
  std::vector<std::vector<int>> panel_ids;
  std::vector<int> node_desc(tb.nodes.size(), -1);
  // a level is eliminated in LDS when all its fronts fit, else by panels
  std::vector<int> level_max_n(max_level + 1, 0);
  for (auto& n : tb.nodes)
    if (!n.leaf) level_max_n[n.level] = std::max(level_max_n[n.level], (int)n.dofs.size());
  long long inv_total = 0;
  long long r_total = 0;
  std::vector<long long> node_r(tb.nodes.size(), -1);
  for (size_t i = 0; i < tb.nodes.size(); ++i) {
    if (tb.nodes[i].leaf) continue;
    node_r[i] = r_total;
    r_total += (long long)tb.nodes[i].dofs.size();
  }
  for (size_t i = 0; i < tb.nodes.size(); ++i) {
    const HNode& n = tb.nodes[i];
    if (n.leaf) continue;
    NodeDesc d{};
    d.f_off = n.f_off;
    d.n = (int)n.dofs.size();
    d.s = n.s;
    d.blocked = level_max_n[n.level] > SMALL_FRONT ? 1 : 0;
    d.inv_off = inv_total;
    d.r_off = node_r[i];
    if (d.blocked)
      inv_total += (long long)((n.s + PANEL_NB - 1) / PANEL_NB) * PANEL_NB * PANEL_NB;
    if (d.n > MAX_FRONT) return fail(c, MRCM_E_UNSUPPORTED, "interface front too large");
    d.map_off = (long long)maps.size();
    d.dof_off = (long long)dofs.size();
    for (int q = 0; q < 2; ++q) {
      const HNode& ch = tb.nodes[n.child[q]];
      d.cr_off[q] = ch.leaf ? -1 : node_r[n.child[q]] + ch.s;
      if (ch.leaf) {
        d.c_off[q] = (long long)ch.sd * c->leaf_block;
        d.c_ld[q] = 4 * g.D + 1;
        d.c_rhs[q] = 4 * g.D;
      } else {
        const int cn = (int)ch.dofs.size();
        d.c_off[q] = ch.f_off + (long long)ch.s * (cn + 1) + ch.s;
        d.c_ld[q] = cn + 1;
        d.c_rhs[q] = cn - ch.s;
      }
    }
    for (int dof : n.dofs) {
      const int ia = tb.schur_index(n.child[0], dof, pos);
      const int ib = tb.schur_index(n.child[1], dof, pos);
      if (ia < 0 && ib < 0) return fail(c, MRCM_E_INVAL, "internal: interface plan is inconsistent");
      maps.push_back(make_int2(ia, ib));
      dofs.push_back(dof);
    }
    node_desc[i] = (int)desc.size();
    desc.push_back(d);
  }
  // algorithmic work of the elimination: per front of n unknowns with s
  // eliminated (and one right-hand side), the extend-add, the LU steps
  // (m multipliers and an m x (m + 1) rank-one update at pivot k, m = n-k-1)
  // and the back substitution of the s eliminated unknowns
  c->iface_flop = 0.0;
  for (const HNode& n : tb.nodes) {
    if (n.leaf) continue;
    const double nn = (double)n.dofs.size(), ss = n.s;
    double f = nn * (nn + 1.0) + 2.0 * ss * (nn - ss) + ss * ss;
    for (int k = 0; k < n.s; ++k) {
      const double m = nn - k - 1.0;
      f += m + 2.0 * m * (m + 1.0);
    }
    c->iface_flop += f;
  }
  for (int lv = 1; lv <= max_level; ++lv) {
    LevelPlan lp{};
    lp.ids_off = (int)ids.size();
    for (size_t i = 0; i < tb.nodes.size(); ++i) {
      const HNode& n = tb.nodes[i];
      if (n.leaf || n.level != lv) continue;
      ids.push_back(node_desc[i]);
      lp.max_n = std::max(lp.max_n, (int)n.dofs.size());
      lp.max_s = std::max(lp.max_s, n.s);
    }
    lp.count = (int)ids.size() - lp.ids_off;
    if (lp.count == 0) continue;
    if (lp.max_s > 2048) return fail(c, MRCM_E_UNSUPPORTED, "interface separator too large");
    lp.small = lp.max_n <= SMALL_FRONT;
    if (!lp.small) {
      for (int k0 = 0; k0 < lp.max_s; k0 += PANEL_NB) {
        PanelLaunch pl{};
        pl.k0 = k0;
        std::vector<int> diag;
        pl.update_off = (int)items.size();
        for (int q = 0; q < lp.count; ++q) {
          const int id = ids[lp.ids_off + q];
          const NodeDesc& d = desc[id];
          if (d.s <= k0) continue;
          diag.push_back(id);
          const int nb = std::min(PANEL_NB, d.s - k0);
          const bool next = d.s > k0 + nb;   // a next panel: its diagonal block gets its own item
          if (next)
            items.push_back(PanelItem{id, k0 + nb, k0 + nb, 2, d.n, d.s, d.f_off, d.inv_off});
          // a rhs column left alone after whole tiles goes with the tile before it
          for (int r = k0 + nb; r < d.n; r += TILE)
            for (int cc = k0 + nb; cc <= d.n; cc += TILE)
              if (cc < d.n || cc == k0 + nb)
                items.push_back(PanelItem{id, r, cc, (next && r == k0 + nb && cc == k0 + nb) ? 1 : 0,
                                          d.n, d.s, d.f_off, d.inv_off});
          if (k0 == 0 && d.n == nb) {
            // the first panel assembles the front; without trailing tiles
            // (which store the panel's rows as they read them) its rows
            // are stored by items of their own
            for (int cc = 0; cc <= d.n; cc += TILE)
              items.push_back(PanelItem{id, 0, cc, 3, d.n, d.s, d.f_off, d.inv_off});
          }
        }
        pl.update_count = (int)items.size() - pl.update_off;
        // the items that update and invert the next diagonal blocks first:
        // they are the critical path of the panel
        std::stable_partition(items.begin() + pl.update_off, items.end(),
                              [](const PanelItem& q) { return q.pad == 2; });
        // then the tiles of each front on one XCD (the work-groups of a
        // launch go to the 8 XCDs in turn), so that the operands they share
        // are fetched into one L2: fronts are dealt to the least loaded XCD,
        // and work-group b takes the next tile of XCD b mod 8 (interface
        // phase about 5 us shorter)
        {
          const auto tiles = std::find_if(items.begin() + pl.update_off, items.end(),
                                          [](const PanelItem& q) { return q.pad != 2; });
          std::vector<std::vector<PanelItem>> xq(8);
          for (auto it = tiles; it != items.end();) {
            auto e = it;   // the items of one front are consecutive
            while (e != items.end() && e->node == it->node) ++e;
            size_t x = 0;
            for (size_t k = 1; k < 8; ++k)
              if (xq[k].size() < xq[x].size()) x = k;
            xq[x].insert(xq[x].end(), it, e);
            it = e;
          }
          std::vector<size_t> pos(8, 0);
          for (auto it = tiles; it != items.end(); ++it) {
            size_t x = (size_t)((it - items.begin()) - pl.update_off) % 8;
            if (pos[x] == xq[x].size())   // that XCD's tiles are all placed
              for (x = 0; pos[x] == xq[x].size(); ++x) {}
            *it = xq[x][pos[x]++];
          }
        }
        pl.diag_count = (int)diag.size();
        panel_ids.push_back(diag);
        pl.diag_off = -1;  // resolved after all level ids are known
        lp.panels.push_back(pl);
      }
    }
    c->levels.push_back(lp);
  }
  // append the per-panel front lists after the per-level lists
  {
    size_t q = 0;
    for (LevelPlan& lp : c->levels)
      for (PanelLaunch& pl : lp.panels) {
        pl.diag_off = (int)ids.size();
        ids.insert(ids.end(), panel_ids[q].begin(), panel_ids[q].end());
        ++q;
      }
  }
  // launches of one solve (run_interface): a level of small fronts takes
  // one, a blocked level one per panel with trailing rows; one back
  // substitution per level; the residual
  c->iface_launches = 1;
  for (const LevelPlan& lp : c->levels) {
    c->iface_launches += 1;
    if (lp.small) c->iface_launches += 1;
    else
      for (const PanelLaunch& pl : lp.panels) c->iface_launches += pl.update_count > 0 ? 1 : 0;
  }
  ALLOC(c, c->tree, total);
  ALLOC(c, c->inv, inv_total);
  ALLOC(c, c->rtree, r_total);
  ALLOC(c, c->rvec, c->n_dof);
  ALLOC(c, c->dx, c->n_dof);
  // the coefficients and corrections of unknowns the plan leaves out stay 0
  HIPCHK(c, hipMemset(c->coef, 0, std::max(c->n_dof, 1) * sizeof(double)));
  HIPCHK(c, hipMemset(c->dx, 0, std::max(c->n_dof, 1) * sizeof(double)));
  ALLOC(c, c->partials, 2 * RESID_WG);
  ALLOC(c, c->d_nodes, desc.size());
  ALLOC(c, c->d_maps, maps.size());
  ALLOC(c, c->d_dofs, dofs.size());
  ALLOC(c, c->d_ids, ids.size());
  ALLOC(c, c->d_lvnodes, ids.size());
  ALLOC(c, c->d_items, items.size());
  HIPCHK(c, hipMemcpy(c->d_nodes, desc.data(), desc.size() * sizeof(NodeDesc), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_maps, maps.data(), maps.size() * sizeof(int2), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_dofs, dofs.data(), dofs.size() * sizeof(int), hipMemcpyHostToDevice));
  HIPCHK(c, hipMemcpy(c->d_ids, ids.data(), ids.size() * sizeof(int), hipMemcpyHostToDevice));
  {
    std::vector<NodeDesc> lv(ids.size());
    for (size_t k = 0; k < ids.size(); ++k) lv[k] = desc[ids[k]];
    HIPCHK(c, hipMemcpy(c->d_lvnodes, lv.data(), lv.size() * sizeof(NodeDesc), hipMemcpyHostToDevice));
  }
  if (!items.empty())
    HIPCHK(c, hipMemcpy(c->d_items, items.data(), items.size() * sizeof(PanelItem), hipMemcpyHostToDevice));
  return MRCM_OK;
}

SubArgs sub_args(const mrcm_ctx* c) {
  SubArgs a{};
  a.g = c->g;
  a.K = c->K;
  a.lam = c->lam;
  a.src = c->src;
  a.rho = c->grav != 0.0 ? c->rho : nullptr;
  a.nact = c->nact;
  a.g.grav = c->grav;
  for (int s = 0; s < 4; ++s) a.bcv[s] = c->bcv[s];
  a.alpha = c->alpha;
  a.basis = c->basis;
  a.X = c->X;
  a.blocks = c->tree;  // the subdomain blocks are the leaves of the interface tree
  a.coef = c->coef;
  a.p_out = c->p;
  a.ux = c->ux;
  a.uy = c->uy;
  a.sub_stats = c->sub_stats;
  a.status = c->status;
  a.fallback = c->fallback;
  a.ir_iters = c->ir_iters;
  a.gate_tol = c->gate_tol;
  a.ir_max = c->ir_max;
  a.ir_tol = c->ir_tol;
  a.scratch = c->scratch;
  a.scratch_stride = c->scratch_stride;
  a.stamps = c->stamps;
  return a;
}

__global__ void zero_int_kernel(int* p) { *p = 0; }

// clears the status words of a solve and stamps its start
__global__ void zero_ints_kernel(int* a, int* b, int* c, unsigned long long* stamps) {
  *a = 0; *b = 0; *c = 0;
  stamp_now(stamps + STAMP_SOLVE);
}

// milliseconds between two phase stamps of the report just read
double stamp_ms(const mrcm_ctx* c, int from, int to) {
  const unsigned long long* s = reinterpret_cast<const unsigned long long*>(c->h_report + STAMP_OFF);
  return s[to] >= s[from] ? (double)(s[to] - s[from]) / c->clock_khz : 0.0;
}

// copy the head of the report block into the pinned host mirror and wait
hipError_t read_report(mrcm_ctx* c) {
  hipError_t e = hipMemcpyAsync(c->h_report, c->report, REPORT_HEAD, hipMemcpyDeviceToHost, c->st);
  if (e != hipSuccess) return e;
  return hipStreamSynchronize(c->st);
}

int run_interface(mrcm_ctx* c) {
  hipStream_t st = c->st;
  // the first launch stamps the start of the interface phase
  unsigned long long* stamp = c->stamps + STAMP_IFACE;
  for (const LevelPlan& lp : c->levels) {
    if (lp.small) {
      HIPCHK(c, launch_front_small(c->d_lvnodes + lp.ids_off, lp.count, lp.max_n, c->tree,
                                   c->d_maps, c->status, stamp, st));
      stamp = nullptr;
      continue;
    }
    // the first panel assembles the fronts and inverts its own diagonal
    // block; each panel inverts the next one
    for (const PanelLaunch& pl : lp.panels)
      if (pl.update_count > 0) {   // the root's last panel has no trailing rows
        HIPCHK(c, launch_front_update(c->d_nodes, c->d_items + pl.update_off, pl.update_count,
                                      pl.k0, c->tree, c->d_maps, c->inv, c->status, stamp, st));
        stamp = nullptr;
      }
  }
  for (auto it = c->levels.rbegin(); it != c->levels.rend(); ++it)
    HIPCHK(c, launch_front_back(c->d_lvnodes + it->ids_off, it->count, it->max_n, c->tree, c->inv, c->d_dofs,
                                nullptr, c->coef, st));
  HIPCHK(c, launch_iface_residual(c->g, c->tree, c->coef, c->rvec, c->partials, c->result + 2,
                                  c->stamps + STAMP_IFACE_END, st));
  return MRCM_OK;
}

// One step of iterative refinement of the interface solution with the
// stored factors: the residual left in rvec by the last residual launch is
// eliminated through the tree into dx, added to the coefficients, and the
// residual is formed again.
int refine_interface(mrcm_ctx* c) {
  hipStream_t st = c->st;
  for (const LevelPlan& lp : c->levels)
    HIPCHK(c, launch_front_rhs(c->d_lvnodes + lp.ids_off, lp.count, lp.max_n, c->tree, c->inv, c->d_maps,
                               c->d_dofs, c->rvec, c->rtree, st));
  for (auto lv = c->levels.rbegin(); lv != c->levels.rend(); ++lv)
    HIPCHK(c, launch_front_back(c->d_lvnodes + lv->ids_off, lv->count, lv->max_n, c->tree, c->inv, c->d_dofs,
                                c->rtree, c->dx, st));
  HIPCHK(c, launch_add(c->coef, c->dx, c->n_dof, st));
  HIPCHK(c, launch_iface_residual(c->g, c->tree, c->coef, c->rvec, c->partials, c->result + 2,
                                  c->stamps + STAMP_IFACE_END, st));
  return MRCM_OK;
}

}  // namespace

extern "C" {

int mrcm_setup(mrcm_ctx** out, const mrcm_grid* g, const double* perm, int32_t sub_nx,
               int32_t sub_ny, int32_t space, int32_t p_dofs, int32_t u_dofs,
               const double* alpha_per_interface, double alpha_scalar, const mrcm_bc* bc,
               const double* source, const mrcm_fluid* fluid, int32_t precision,
               void* hip_stream) {
  if (!out) return MRCM_E_INVAL;
  *out = nullptr;
  if (!g || !perm || !bc || !fluid) return MRCM_E_INVAL;
  if (g->nx <= 0 || g->ny <= 0 || !finite_pos(g->lx) || !finite_pos(g->ly)) return MRCM_E_INVAL;
  if (sub_nx != sub_ny) return MRCM_E_UNSUPPORTED;
  const int M = sub_nx;
  if (!(M == 4 || M == 8 || M == 16 || M == 32)) return MRCM_E_UNSUPPORTED;
  if (g->nx % M || g->ny % M) return MRCM_E_INVAL;
  if (space == MRCM_SPACE_LINEAR || space == MRCM_SPACE_EDGE_SOLUTION) {
    if (p_dofs != 2 || u_dofs != 2) return MRCM_E_INVAL;
  } else if (space == MRCM_SPACE_FULL) {
    if (p_dofs != M || u_dofs != M) return MRCM_E_INVAL;
  } else if (space == MRCM_SPACE_PHYSICS) {
    if (p_dofs != PHYS_P || u_dofs != PHYS_U) return MRCM_E_INVAL;
  } else {
    return MRCM_E_INVAL;
  }
  if (precision != MRCM_PREC_FP64 && precision != MRCM_PREC_FP32_IR &&
      precision != MRCM_PREC_SURROGATE)
    return MRCM_E_INVAL;
  if (precision == MRCM_PREC_FP32_IR && !local_fp32_supported(M, p_dofs + u_dofs, p_dofs))
    return MRCM_E_UNSUPPORTED;
  if (precision == MRCM_PREC_SURROGATE && !(M == 16 && p_dofs == 2 && u_dofs == 2))
    return MRCM_E_UNSUPPORTED;
  if (!finite_pos(fluid->mu_w) || !finite_pos(fluid->mu_o)) return MRCM_E_INVAL;
  for (int s = 0; s < 4; ++s)
    if (bc->kind[s] != MRCM_BC_NEUMANN && bc->kind[s] != MRCM_BC_DIRICHLET) return MRCM_E_INVAL;
  const size_t ncell = (size_t)g->nx * g->ny;
  for (size_t i = 0; i < ncell; ++i)
    if (!finite_pos(perm[i])) return MRCM_E_INVAL;
  const int SX = g->nx / M, SY = g->ny / M;
  const int n_iface = (SX - 1) * SY + SX * (SY - 1);
  if (alpha_per_interface) {
    for (int e = 0; e < n_iface; ++e)
      if (!finite_pos(alpha_per_interface[e])) return MRCM_E_INVAL;
  } else if (!finite_pos(alpha_scalar)) {
    return MRCM_E_INVAL;
  }
  if (!local_supported(M, p_dofs + u_dofs)) return MRCM_E_UNSUPPORTED;
  for (int s = 0; s < 4; ++s) {
    const int n = s < 2 ? g->ny : g->nx;
    if (bc->value[s])
      for (int i = 0; i < n; ++i)
        if (!isfinite(bc->value[s][i])) return MRCM_E_INVAL;
  }
  if (source)
    for (size_t i = 0; i < ncell; ++i)
      if (!isfinite(source[i])) return MRCM_E_INVAL;

  mrcm_ctx* c = new (std::nothrow) mrcm_ctx();
  if (!c) return MRCM_E_NOMEM;
  Geo& G = c->g;
  G.nx = g->nx; G.ny = g->ny; G.M = M; G.SX = SX; G.SY = SY;
  G.nV = (SX - 1) * SY; G.n_sub = SX * SY;
  G.nP = p_dofs; G.nU = u_dofs; G.D = p_dofs + u_dofs;
  G.hx = g->lx / g->nx; G.hy = g->ly / g->ny;
  G.tfx = G.hy / (0.5 * G.hx); G.tfy = G.hx / (0.5 * G.hy);
  bool any_dir = false;
  for (int s = 0; s < 4; ++s) { G.kind[s] = bc->kind[s]; any_dir |= bc->kind[s] == MRCM_BC_DIRICHLET; }
  G.gauge = any_dir ? 0 : 1;
  G.prec = precision;
  {
    const char* gen = getenv("MRCM_GENERIC_KERNELS");
    G.generic = (gen && gen[0] == '1') ? 1 : 0;
  }
  c->precision = precision;
  c->ir_max = LOCAL_IR_MAX;
  c->ir_tol = LOCAL_IR_TOL;
  c->iface_ir_max = IFACE_IR_MAX;
  c->iface_ir_tol = precision == MRCM_PREC_FP32_IR ? IFACE_IR_TOL_FP32 : IFACE_IR_TOL_FP64;
  c->iface_fail_tol = IFACE_FAIL_TOL;
  c->space = space;
  c->mu_w = fluid->mu_w;
  c->mu_o = fluid->mu_o;
  c->n_dof = n_iface * G.D;
  c->R = 1 + 4 * G.D;

  int rc = MRCM_OK;
  auto setup_body = [&]() -> int {
    if (hip_stream) {
      c->st = (hipStream_t)hip_stream;
    } else {
      HIPCHK(c, hipStreamCreate(&c->st));
      c->own_stream = true;
    }
    for (int i = 0; i < 3; ++i) HIPCHK(c, hipEventCreate(&c->ev[i]));
    ALLOC(c, c->K, ncell);
    ALLOC(c, c->lam, ncell);
    ALLOC(c, c->stage, ncell);
    if (source) ALLOC(c, c->src, ncell);
    for (int s = 0; s < 4; ++s) ALLOC(c, c->bcv[s], s < 2 ? G.ny : G.nx);
    ALLOC(c, c->alpha, n_iface);
    ALLOC(c, c->basis, (size_t)std::max(n_iface, 1) * G.D * M);
    ALLOC(c, c->X, (size_t)G.n_sub * M * M * c->R);
    ALLOC(c, c->coef, std::max(c->n_dof, 1));
    ALLOC(c, c->p, ncell);
    ALLOC(c, c->ux, (size_t)(G.nx + 1) * G.ny);
    ALLOC(c, c->uy, (size_t)G.nx * (G.ny + 1));
    ALLOC(c, c->sub_stats, 3 * G.n_sub);
    ALLOC(c, c->report, RESULT_N + (G.n_sub + 4 + 1) / 2);
    c->result = c->report;
    c->status = reinterpret_cast<int*>(c->report + RESULT_N);
    c->stamps = reinterpret_cast<unsigned long long*>(c->report + STAMP_OFF);
    {
      int dev = 0, khz = 0;
      HIPCHK(c, hipGetDevice(&dev));
      HIPCHK(c, hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev));
      if (khz <= 0) return fail(c, MRCM_E_HIP, "device reports no wall clock rate");
      c->clock_khz = khz;
    }
    c->ir_iters = c->status + 1;
    c->fallback = c->status + 2;
    {
      void* h = nullptr;
      HIPCHK(c, hipHostMalloc(&h, REPORT_HEAD, hipHostMallocDefault));
      c->h_report = static_cast<double*>(h);
    }
    {
      // transport work arrays: face couplings, x, r, r^, 2 p, 2 v, q, t
      ALLOC(c, c->tr.cfx, (size_t)(G.nx + 1) * G.ny);
      ALLOC(c, c->tr.cfy, (size_t)G.nx * (G.ny + 1));
      double** vecs[] = {&c->tr.x, &c->tr.r, &c->tr.rh, &c->tr.p[0], &c->tr.p[1], &c->tr.v[0],
                         &c->tr.v[1], &c->tr.q, &c->tr.t};
      for (double** v : vecs) ALLOC(c, *v, ncell);
      const int nb = transport_blocks(G.nx, G.ny);
      for (int k = 0; k < 3; ++k) ALLOC(c, c->tr.part[k], 4 * (size_t)nb);
      ALLOC(c, c->tr.scal, TS_N);
      ALLOC(c, c->s_prev, ncell);
      void* h = nullptr;
      HIPCHK(c, hipHostMalloc(&h, TS_N * sizeof(double), hipHostMallocDefault));
      c->h_tscal = static_cast<double*>(h);
    }
    c->scratch_stride = local_scratch_doubles(G);
    if (c->scratch_stride > 0) ALLOC(c, c->scratch, (size_t)G.n_sub * c->scratch_stride);
    if (precision == MRCM_PREC_SURROGATE) {
      const size_t pix = (size_t)G.n_sub * M * M;
      ALLOC(c, c->s_p32, cnn::n_params());
      ALLOC(c, c->s_wb, cnn::n_params());
      ALLOC(c, c->s_in, pix * 8);
      ALLOC(c, c->s_pred, pix * 16);
    }
    HIPCHK(c, hipMemcpy(c->K, perm, ncell * sizeof(double), hipMemcpyHostToDevice));
    {
      std::vector<double> ones(ncell, 1.0);
      HIPCHK(c, hipMemcpy(c->lam, ones.data(), ncell * sizeof(double), hipMemcpyHostToDevice));
    }
    if (source) HIPCHK(c, hipMemcpy(c->src, source, ncell * sizeof(double), hipMemcpyHostToDevice));
    for (int s = 0; s < 4; ++s) {
      const int n = s < 2 ? G.ny : G.nx;
      std::vector<double> v(n, 0.0);
      if (bc->value[s]) std::copy(bc->value[s], bc->value[s] + n, v.begin());
      HIPCHK(c, hipMemcpy(c->bcv[s], v.data(), n * sizeof(double), hipMemcpyHostToDevice));
    }
    std::vector<double> al(std::max(n_iface, 1), alpha_scalar);
    if (alpha_per_interface) std::copy(alpha_per_interface, alpha_per_interface + n_iface, al.begin());
    HIPCHK(c, hipMemcpy(c->alpha, al.data(), al.size() * sizeof(double), hipMemcpyHostToDevice));
    // interface functions, rows [psi_0.., phi_0..] per interface; the
    // channels of every interface (adaptive alpha)
    std::vector<double> bs((size_t)std::max(n_iface, 1) * G.D * M, 0.0);
    std::vector<double> klo(M), khi(M), tf(M);
    std::vector<int2> nact(std::max(n_iface, 1), make_int2(0, 0));
    c->has_channel.assign(std::max(n_iface, 1), 0);
    for (int e = 0; e < n_iface; ++e) {
      double* b = bs.data() + (size_t)e * G.D * M;
      for (int t = 0; t < M; ++t) {
        size_t cl, ch;
        if (e < G.nV) {
          const int J = e / (SX - 1), I = e % (SX - 1);
          const int i = (I + 1) * M, j = J * M + t;
          cl = (size_t)j * G.nx + i - 1;
          ch = (size_t)j * G.nx + i;
        } else {
          const int h = e - G.nV, J = h / SX, I = h % SX;
          const int j = (J + 1) * M, i = I * M + t;
          cl = (size_t)(j - 1) * G.nx + i;
          ch = (size_t)j * G.nx + i;
        }
        klo[t] = perm[cl];
        khi[t] = perm[ch];
        tf[t] = hmean(klo[t], khi[t]);
      }
      {
        std::vector<Run> chn, bar;
        classify_faces(tf, chn, bar);
        c->has_channel[e] = !chn.empty();
      }
      if (space == MRCM_SPACE_PHYSICS) {
        physics_space(tf, b, M, nact[e].x, nact[e].y);
      } else if (space == MRCM_SPACE_LINEAR) {
        for (int t = 0; t < M; ++t) {
          const double xi = (t + 0.5) / M;
          b[0 * M + t] = 1.0 - xi;
          b[1 * M + t] = xi;
          b[2 * M + t] = 1.0 - xi;
          b[3 * M + t] = xi;
        }
      } else if (space == MRCM_SPACE_FULL) {
        for (int k = 0; k < M; ++k) {
          b[k * M + k] = 1.0;
          b[(M + k) * M + k] = 1.0;
        }
      } else {
        edge_solution(klo, khi, b, M);
      }
    }
    HIPCHK(c, hipMemcpy(c->basis, bs.data(), bs.size() * sizeof(double), hipMemcpyHostToDevice));
    if (space == MRCM_SPACE_PHYSICS) {
      ALLOC(c, c->nact, nact.size());
      HIPCHK(c, hipMemcpy(c->nact, nact.data(), nact.size() * sizeof(int2), hipMemcpyHostToDevice));
      c->h_nact = nact;
    }
    int r = build_plan(c);
    if (r != MRCM_OK) return r;
    r = bind_static_scratch(c);
    if (r != MRCM_OK) return r;
    HIPCHK(c, hipDeviceSynchronize());
    return MRCM_OK;
  };
  rc = setup_body();
  if (rc != MRCM_OK) {
    fprintf(stderr, "mrcm_setup: %s\n", c->err.c_str());
    mrcm_destroy(c);
    return rc;
  }
  *out = c;
  return MRCM_OK;
}

namespace {

// total mobility (and, with gravity, lambda_g / lambda) from device values
int mobility_enqueue(mrcm_ctx* c, const double* src, int32_t values_are_lambda) {
  const size_t n = (size_t)c->g.nx * c->g.ny;
  if (c->grav != 0.0) {
    HIPCHK(c, launch_mobility_gravity(src, c->lam, c->rho, n, c->mu_w, c->mu_o, c->rho_w, c->rho_o, c->st));
    c->rho_valid = true;
    return MRCM_OK;
  }
  HIPCHK(c, launch_mobility(src, c->lam, n, values_are_lambda ? 0 : 1, c->mu_w, c->mu_o, c->st));
  return MRCM_OK;
}

int gravity_check(mrcm_ctx* c, int32_t values_are_lambda) {
  if (c->grav != 0.0 && values_are_lambda)
    return fail(c, MRCM_E_INVAL, "the gravity variant takes the saturation (lambda_g / lambda needs it), "
                                 "not the total mobility");
  return MRCM_OK;
}

}  // namespace

int mrcm_update_mobility(mrcm_ctx* c, const double* values, int32_t values_are_lambda,
                         int32_t on_device) {
  if (!c) return MRCM_E_INVAL;
  if (!values) return fail(c, MRCM_E_INVAL, "values is NULL");
  int r = gravity_check(c, values_are_lambda);
  if (r != MRCM_OK) return r;
  const size_t n = (size_t)c->g.nx * c->g.ny;
  const double* src = values;
  if (!on_device) {
    HIPCHK(c, hipMemcpyAsync(c->stage, values, n * sizeof(double), hipMemcpyHostToDevice, c->st));
    src = c->stage;
  }
  r = mobility_enqueue(c, src, values_are_lambda);
  if (r != MRCM_OK) return r;
  if (!on_device) HIPCHK(c, hipStreamSynchronize(c->st));  // host buffer may be reused on return
  c->solved = false;
  return MRCM_OK;
}

int mrcm_set_adaptive_alpha(mrcm_ctx* c, double alpha_channel, double alpha_other) {
  if (!c) return MRCM_E_INVAL;
  if (!finite_pos(alpha_channel) || !finite_pos(alpha_other))
    return fail(c, MRCM_E_INVAL, "mrcm_set_adaptive_alpha: values must be finite and > 0");
  const int n_iface = (c->g.SX - 1) * c->g.SY + c->g.SX * (c->g.SY - 1);
  if (n_iface == 0) return MRCM_OK;
  std::vector<double> al(n_iface);
  for (int e = 0; e < n_iface; ++e) al[e] = c->has_channel[e] ? alpha_channel : alpha_other;
  HIPCHK(c, hipStreamSynchronize(c->st));   // no kernel of the context still reads alpha
  HIPCHK(c, hipMemcpy(c->alpha, al.data(), n_iface * sizeof(double), hipMemcpyHostToDevice));
  c->solved = false;
  return MRCM_OK;
}

int mrcm_set_gravity(mrcm_ctx* c, double gravity, double rho_w, double rho_o) {
  if (!c) return MRCM_E_INVAL;
  if (!isfinite(gravity) || !isfinite(rho_w) || !isfinite(rho_o))
    return fail(c, MRCM_E_INVAL, "mrcm_set_gravity: values must be finite");
  if (gravity != 0.0 && c->precision == MRCM_PREC_SURROGATE)
    return fail(c, MRCM_E_UNSUPPORTED, "mrcm_set_gravity: the surrogate precision has no gravity variant");
  if (gravity != 0.0 && !c->rho) {
    int r = dev_alloc(c, &c->rho, (size_t)c->g.nx * c->g.ny);
    if (r != MRCM_OK) return r;
  }
  c->grav = gravity;
  c->rho_w = rho_w;
  c->rho_o = rho_o;
  c->g.grav = gravity;
  c->rho_valid = false;
  c->solved = false;
  return MRCM_OK;
}

namespace {

// The work of one solve, enqueued on the context's stream: local solves
// (with the surrogate precision `pred`, device, may be NULL, replaces the
// network's output), interface solve and its residual check.
int solve_enqueue(mrcm_ctx* c, const float* pred) {
  hipStream_t st = c->st;
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(1), 0, st, c->status, c->fallback, c->ir_iters,
                     c->stamps);
  HIPCHK(c, hipGetLastError());
  // the phases are timed by the kernels' clock stamps; events (each a packet
  // that drains the stream) only where no kernel marks the boundary: the
  // surrogate's gate, and the end of the local phase when there is no
  // interface system
  const bool ev_local = c->n_dof == 0, ev_gate = c->precision == MRCM_PREC_SURROGATE;
  if (ev_local || ev_gate) HIPCHK(c, hipEventRecord(c->ev[0], st));
  SubArgs a = sub_args(c);
  if (c->precision == MRCM_PREC_SURROGATE) {
    // network inference and residual gate, then the FP64 kernel on the
    // subdomains the gate rejected
    const int n = c->g.n_sub;
    if (!pred) {
      HIPCHK(c, launch_surrogate_inputs(a, c->s_in, st));
      HIPCHK(c, cnn::forward_fused(c->s_in, c->s_wb, c->s_p32, c->s_pred, n, st));
      pred = c->s_pred;
    }
    HIPCHK(c, launch_surrogate_gate(a, pred, st));
    HIPCHK(c, hipEventRecord(c->ev[2], st));
    HIPCHK(c, launch_basis_m16d4_list(a, st));
  } else {
    HIPCHK(c, launch_local_basis(a, st));
  }
  if (ev_local) HIPCHK(c, hipEventRecord(c->ev[1], st));
  if (c->n_dof > 0) {
    int r = run_interface(c);
    if (r != MRCM_OK) return r;
  }
  return MRCM_OK;
}

// Residual of the interface solve in the report just read: above ir_tol of
// the right-hand side (high contrast with non-polynomial spaces makes the
// system ill-conditioned) the solve is refined, each step checked at a
// synchronisation of its own; well-conditioned solves pay nothing.
bool iface_above(const mrcm_ctx* c, double tol) {
  return c->n_dof > 0 && !(c->h_report[2] <= tol * c->h_report[3]);
}

bool needs_refinement(const mrcm_ctx* c) {
  return c->iface_ir < c->iface_ir_max && iface_above(c, c->iface_ir_tol);
}

// Statistics and status of a solve whose report has been read (and
// refined while needed).
int solve_finish(mrcm_ctx* c) {
  while (needs_refinement(c)) {
    int r = refine_interface(c);
    if (r != MRCM_OK) return r;
    HIPCHK(c, read_report(c));
    c->iface_ir += 1;
  }
  const int* hi = reinterpret_cast<const int*>(c->h_report + RESULT_N);
  const int status = hi[0], iters = hi[1], nfb = hi[2];
  const double res[2] = {c->h_report[2], c->h_report[3]};
  if (c->n_dof > 0) {
    c->stats.ms_local = stamp_ms(c, STAMP_SOLVE, STAMP_IFACE);
    c->stats.ms_interface = stamp_ms(c, STAMP_IFACE, STAMP_IFACE_END);
  } else {
    float t = 0.f;
    (void)hipEventElapsedTime(&t, c->ev[0], c->ev[1]);
    c->stats.ms_local = t;
    c->stats.ms_interface = 0.0;
  }
  c->stats.ms_surrogate = 0.0;
  if (c->precision == MRCM_PREC_SURROGATE) {
    float ts = 0.f;
    (void)hipEventElapsedTime(&ts, c->ev[0], c->ev[2]);
    c->stats.ms_surrogate = ts;
  }
  c->stats.interface_residual = res[1] > 0.0 ? res[0] / res[1] : 0.0;
  c->stats.fallbacks = c->g.prec != 0 ? nfb : 0;
  c->stats.interface_ir_steps = c->iface_ir;
  c->stats.ir_iters_max = c->g.prec != 0 ? iters : 0;
  if (status & ST_BAD_LAMBDA) return fail(c, MRCM_E_INVAL, "mobility not finite and positive");
  if (status & (ST_LOCAL_PIVOT | ST_IFACE_PIVOT))
    return fail(c, MRCM_E_NOT_SPD, "non-positive or zero pivot in the elimination");
  if (iface_above(c, c->iface_fail_tol)) {
    // the interface elimination does not pivot: a nearly singular pivot
    // shows as a residual that refinement does not bring down
    char msg[160];
    snprintf(msg, sizeof msg, "interface solve: residual %.3e of the right-hand side after %d "
             "refinement steps (failure above %.3e)", c->stats.interface_residual, c->iface_ir,
             c->iface_fail_tol);
    return fail(c, MRCM_E_NO_CONV, msg);
  }
  c->solved = true;
  return MRCM_OK;
}

int solve_impl(mrcm_ctx* c, const float* pred) {
  c->solved = false;
  int r = solve_enqueue(c, pred);
  if (r != MRCM_OK) return r;
  HIPCHK(c, read_report(c));
  c->iface_ir = 0;
  return solve_finish(c);
}

// The fine-scale reconstruction, enqueued: stitch and flux statistics, and
// the copies of host outputs.  The stitch's pivot flag joins the solve's
// status word (cleared by the solve).
int flux_enqueue(mrcm_ctx* c, double* p, double* ux, double* uy, int32_t on_device,
                 double* sub_stats = nullptr, double* result = nullptr) {
  hipStream_t st = c->st;
  const Geo& G = c->g;
  SubArgs a = sub_args(c);
  // per-subdomain statistics and their reduction: the context's buffers, or
  // the static scratch (mrcm_fine_flux_static)
  if (sub_stats) a.sub_stats = sub_stats;
  if (!result) result = c->result;
  // device outputs are written by the kernels in place; host outputs are
  // copied from the context's buffers
  if (on_device) {
    if (p) a.p_out = p;
    if (ux) a.ux = ux;
    if (uy) a.uy = uy;
  }
  HIPCHK(c, launch_stitch(a, st));
  HIPCHK(c, launch_finish_flux(a, result, st));
  const size_t ncell = (size_t)G.nx * G.ny;
  if (!on_device) {
    const hipMemcpyKind kind = hipMemcpyDeviceToHost;
    if (p) HIPCHK(c, hipMemcpyAsync(p, c->p, ncell * sizeof(double), kind, st));
    if (ux) HIPCHK(c, hipMemcpyAsync(ux, c->ux, (size_t)(G.nx + 1) * G.ny * sizeof(double), kind, st));
    if (uy) HIPCHK(c, hipMemcpyAsync(uy, c->uy, (size_t)G.nx * (G.ny + 1) * sizeof(double), kind, st));
  }
  return MRCM_OK;
}

// after the report of a reconstruction has been read
int flux_finish(mrcm_ctx* c, double* max_cell_imbalance) {
  const int status = reinterpret_cast<const int*>(c->h_report + RESULT_N)[0];
  c->stats.ms_flux = stamp_ms(c, STAMP_FLUX, STAMP_FLUX_END);
  if (max_cell_imbalance) *max_cell_imbalance = c->h_report[0];
  if (status & ST_STITCH_PIVOT) return fail(c, MRCM_E_NOT_SPD, "non-positive pivot in the stitch re-solve");
  return MRCM_OK;
}

}  // namespace

int mrcm_solve(mrcm_ctx* c) {
  if (!c) return MRCM_E_INVAL;
  if (c->precision == MRCM_PREC_SURROGATE && !c->s_ready)
    return fail(c, MRCM_E_STATE, "surrogate precision: mrcm_set_surrogate was not called");
  if (c->grav != 0.0 && !c->rho_valid)
    return fail(c, MRCM_E_STATE, "gravity: no saturation given since mrcm_set_gravity");
  return solve_impl(c, nullptr);
}

int mrcm_solve_with_predictions(mrcm_ctx* c, const float* predictions) {
  if (!c) return MRCM_E_INVAL;
  if (!predictions) return fail(c, MRCM_E_INVAL, "predictions is NULL");
  if (c->precision != MRCM_PREC_SURROGATE)
    return fail(c, MRCM_E_STATE, "context was not set up with MRCM_PREC_SURROGATE");
  return solve_impl(c, predictions);
}

int mrcm_fine_flux(mrcm_ctx* c, double* p, double* ux, double* uy, int32_t on_device,
                   double* max_cell_imbalance) {
  if (!c) return MRCM_E_INVAL;
  if (!c->solved) return fail(c, MRCM_E_STATE, "fine_flux called before a successful solve");
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, c->st, c->status);
  HIPCHK(c, hipGetLastError());
  int r = flux_enqueue(c, p, ux, uy, on_device);
  if (r != MRCM_OK) return r;
  HIPCHK(c, read_report(c));
  return flux_finish(c, max_cell_imbalance);
}

int mrcm_fine_flux_static(mrcm_ctx* c, double* p, double* ux, double* uy, int32_t on_device,
                          double* max_cell_imbalance) {
  if (!c) return MRCM_E_INVAL;
  if (!c->solved) return fail(c, MRCM_E_STATE, "fine_flux called before a successful solve");
  if (c->g.n_sub > STATIC_MAX_SUB)
    return fail(c, MRCM_E_INVAL, "mrcm_fine_flux_static: more than 65536 subdomains (its scratch "
                                 "holds 3 doubles per subdomain for at most 65536)");
  if (!c->static_scratch) return fail(c, MRCM_E_STATE, "static scratch not bound to this device");
  double* sub_stats = c->static_scratch;
  double* result = c->static_scratch + 3 * (size_t)STATIC_MAX_SUB;
  hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, c->st, c->status);
  HIPCHK(c, hipGetLastError());
  int r = flux_enqueue(c, p, ux, uy, on_device, sub_stats, result);
  if (r != MRCM_OK) return r;
  // the report head (status word, phase stamps), then the two reduced
  // values from the scratch over its first two slots
  HIPCHK(c, hipMemcpyAsync(c->h_report, c->report, REPORT_HEAD, hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipMemcpyAsync(c->h_report, result, 2 * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return flux_finish(c, max_cell_imbalance);
}

int mrcm_step(mrcm_ctx* c, const double* values, int32_t values_are_lambda, int32_t values_on_device,
              double* p, double* ux, double* uy, int32_t outputs_on_device, double* max_cell_imbalance) {
  if (!c) return MRCM_E_INVAL;
  if (c->precision == MRCM_PREC_SURROGATE && !c->s_ready)
    return fail(c, MRCM_E_STATE, "surrogate precision: mrcm_set_surrogate was not called");
  if (values) {
    int r = gravity_check(c, values_are_lambda);
    if (r != MRCM_OK) return r;
    const size_t n = (size_t)c->g.nx * c->g.ny;
    const double* src = values;
    if (!values_on_device) {   // the host array is read before the call returns
      HIPCHK(c, hipMemcpyAsync(c->stage, values, n * sizeof(double), hipMemcpyHostToDevice, c->st));
      src = c->stage;
    }
    r = mobility_enqueue(c, src, values_are_lambda);
    if (r != MRCM_OK) return r;
  }
  if (c->grav != 0.0 && !c->rho_valid)
    return fail(c, MRCM_E_STATE, "gravity: no saturation given since mrcm_set_gravity");
  c->solved = false;
  int r = solve_enqueue(c, nullptr);
  if (r != MRCM_OK) return r;
  if (c->step_refined) {
    // the last step refined its interface solve: this one most likely will
    // too, so the reconstruction waits for the refined solution instead of
    // being enqueued (and redone) on the unrefined one
    HIPCHK(c, read_report(c));
    c->iface_ir = 0;
    r = solve_finish(c);
    if (r != MRCM_OK) return r;
    c->step_refined = c->iface_ir > 0;
    r = flux_enqueue(c, p, ux, uy, outputs_on_device);
    if (r != MRCM_OK) return r;
    HIPCHK(c, read_report(c));
    return flux_finish(c, max_cell_imbalance);
  }
  // the reconstruction is enqueued before the solve's status is known; one
  // synchronisation reads both reports
  r = flux_enqueue(c, p, ux, uy, outputs_on_device);
  if (r != MRCM_OK) return r;
  HIPCHK(c, read_report(c));
  c->iface_ir = 0;
  c->step_refined = needs_refinement(c);
  if (needs_refinement(c)) {
    // refine (solve_finish synchronises per step), then reconstruct again
    r = solve_finish(c);
    if (r != MRCM_OK) return r;
    hipLaunchKernelGGL(zero_int_kernel, dim3(1), dim3(1), 0, c->st, c->status);
    HIPCHK(c, hipGetLastError());
    r = flux_enqueue(c, p, ux, uy, outputs_on_device);
    if (r != MRCM_OK) return r;
    HIPCHK(c, read_report(c));
    return flux_finish(c, max_cell_imbalance);
  }
  r = solve_finish(c);
  if (r != MRCM_OK) return r;
  return flux_finish(c, max_cell_imbalance);
}

int mrcm_get_stats(const mrcm_ctx* c, mrcm_stats* s) {
  if (!c || !s) return MRCM_E_INVAL;
  *s = c->stats;
  s->n_sub = c->g.n_sub;
  s->n_dof = c->n_dof;
  s->interface_gflop = c->iface_flop * 1e-9;
  s->interface_launches = c->iface_launches;
  return MRCM_OK;
}

int mrcm_get_sizes(const mrcm_ctx* c, int32_t* n_dof, int32_t* n_sub, int32_t* n_cols) {
  if (!c) return MRCM_E_INVAL;
  if (n_dof) *n_dof = c->n_dof;
  if (n_sub) *n_sub = c->g.n_sub;
  if (n_cols) *n_cols = c->R;
  return MRCM_OK;
}

int mrcm_get_interface_solution(mrcm_ctx* c, double* coeffs) {
  if (!c || !coeffs) return MRCM_E_INVAL;
  if (!c->solved) return fail(c, MRCM_E_STATE, "no solve yet");
  if (c->n_dof == 0) return MRCM_OK;
  HIPCHK(c, hipMemcpyAsync(coeffs, c->coef, c->n_dof * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return MRCM_OK;
}

int mrcm_get_local_blocks(mrcm_ctx* c, double* blocks) {
  if (!c || !blocks) return MRCM_E_INVAL;
  if (!c->solved) return fail(c, MRCM_E_STATE, "no solve yet");
  HIPCHK(c, hipMemcpyAsync(blocks, c->tree, (size_t)c->g.n_sub * c->leaf_block * sizeof(double),
                           hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return MRCM_OK;
}

int mrcm_get_basis(mrcm_ctx* c, double* basis) {
  if (!c || !basis) return MRCM_E_INVAL;
  if (!c->solved) return fail(c, MRCM_E_STATE, "no solve yet");
  const size_t n = (size_t)c->g.n_sub * c->g.M * c->g.M * c->R;
  HIPCHK(c, hipMemcpyAsync(basis, c->X, n * sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return MRCM_OK;
}

static bool surrogate_shape(const mrcm_ctx* c) {
  return c->g.M == 16 && c->g.nP == 2 && c->g.nU == 2;
}

int mrcm_surrogate_inputs(mrcm_ctx* c, void* inputs) {
  if (!c) return MRCM_E_INVAL;
  if (!inputs) return fail(c, MRCM_E_INVAL, "inputs is NULL");
  if (!surrogate_shape(c)) return fail(c, MRCM_E_UNSUPPORTED, "surrogate needs 16x16 subdomains, 2+2 dofs");
  HIPCHK(c, launch_surrogate_inputs(sub_args(c), (short*)inputs, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return MRCM_OK;
}

int mrcm_surrogate_targets(mrcm_ctx* c, float* targets) {
  if (!c) return MRCM_E_INVAL;
  if (!targets) return fail(c, MRCM_E_INVAL, "targets is NULL");
  if (!surrogate_shape(c)) return fail(c, MRCM_E_UNSUPPORTED, "surrogate needs 16x16 subdomains, 2+2 dofs");
  if (!c->solved) return fail(c, MRCM_E_STATE, "no solve yet");
  HIPCHK(c, launch_surrogate_targets(sub_args(c), targets, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  return MRCM_OK;
}

int mrcm_set_gate_tolerance(mrcm_ctx* c, double tol) {
  if (!c) return MRCM_E_INVAL;
  if (!(tol > 0.0) || !isfinite(tol)) return fail(c, MRCM_E_INVAL, "gate tolerance must be finite and > 0");
  if (c->precision != MRCM_PREC_SURROGATE)
    return fail(c, MRCM_E_STATE, "context was not set up with MRCM_PREC_SURROGATE");
  c->gate_tol = tol;
  return MRCM_OK;
}

int mrcm_set_refinement(mrcm_ctx* c, int32_t max_steps, double tol) {
  if (!c) return MRCM_E_INVAL;
  if (max_steps < 0 || max_steps > 64 || !(tol > 0.0) || !(tol < 1.0))
    return fail(c, MRCM_E_INVAL, "refinement: 0 <= max_steps <= 64 and 0 < tol < 1 required");
  if (c->precision != MRCM_PREC_FP32_IR)
    return fail(c, MRCM_E_STATE, "context was not set up with MRCM_PREC_FP32_IR");
  c->ir_max = max_steps;
  c->ir_tol = tol;
  return MRCM_OK;
}

int mrcm_set_interface_refinement(mrcm_ctx* c, int32_t max_steps, double tol, double fail_tol) {
  if (!c) return MRCM_E_INVAL;
  if (max_steps < 0 || max_steps > 16 || !(tol > 0.0) || !(tol < 1.0) || !(fail_tol > 0.0) ||
      !(fail_tol < 1.0))
    return fail(c, MRCM_E_INVAL, "interface refinement: 0 <= max_steps <= 16, 0 < tol < 1 and "
                                 "0 < fail_tol < 1 required");
  c->iface_ir_max = max_steps;
  c->iface_ir_tol = tol;
  c->iface_fail_tol = fail_tol;
  return MRCM_OK;
}

int mrcm_set_surrogate(mrcm_ctx* c, mrcm_cnn* net) {
  if (!c) return MRCM_E_INVAL;
  if (!net) return fail(c, MRCM_E_INVAL, "net is NULL");
  if (c->precision != MRCM_PREC_SURROGATE)
    return fail(c, MRCM_E_STATE, "context was not set up with MRCM_PREC_SURROGATE");
  HIPCHK(c, hipStreamSynchronize(cnn::stream_of(net)));
  HIPCHK(c, hipMemcpyAsync(c->s_p32, cnn::params_of(net), cnn::n_params() * sizeof(float),
                           hipMemcpyDeviceToDevice, c->st));
  HIPCHK(c, cnn::cast(c->s_p32, c->s_wb, c->st));
  HIPCHK(c, hipStreamSynchronize(c->st));
  c->s_ready = true;
  return MRCM_OK;
}

namespace {

int transport_check(mrcm_ctx* c, const double* s_old, double* s_new, const double* ux,
                    const double* uy, double dt, double s_inflow, double eta, int32_t max_newton) {
  if (c->grav != 0.0)
    return fail(c, MRCM_E_UNSUPPORTED, "transport: no gravity segregation term (set gravity to 0)");
  if (!s_old || !s_new || !ux || !uy) return fail(c, MRCM_E_INVAL, "transport: NULL array");
  if (s_old == s_new) return fail(c, MRCM_E_INVAL, "transport: s_new must not alias s_old");
  if (!(dt > 0.0) || !isfinite(dt)) return fail(c, MRCM_E_INVAL, "transport: dt must be finite and > 0");
  if (!(s_inflow >= 0.0 && s_inflow <= 1.0)) return fail(c, MRCM_E_INVAL, "transport: 0 <= s_inflow <= 1");
  if (!(eta > 0.0) || !isfinite(eta)) return fail(c, MRCM_E_INVAL, "transport: eta must be finite and > 0");
  if (max_newton < 1 || max_newton > 1000) return fail(c, MRCM_E_INVAL, "transport: 1 <= max_newton <= 1000");
  return MRCM_OK;
}

int transport_impl(mrcm_ctx* c, const double* s_old, double* s_new, const double* ux,
                   const double* uy, double dt, double s_inflow, double eta, int32_t max_newton,
                   mrcm_transport_stats* stats) {
  const auto t0 = std::chrono::steady_clock::now();
  const Geo& G = c->g;
  const size_t n = (size_t)G.nx * G.ny;
  TransportArgs a = c->tr;
  a.nx = G.nx;
  a.ny = G.ny;
  a.hx = G.hx;
  a.hy = G.hy;
  a.V = G.hx * G.hy;
  a.c = dt / a.V;
  a.M = c->mu_o / c->mu_w;
  {
    const double w = a.M * s_inflow * s_inflow, o = (1.0 - s_inflow) * (1.0 - s_inflow);
    a.fin = w / (w + o);
  }
  a.tol2 = TRANSPORT_LIN_TOL * TRANSPORT_LIN_TOL;
  a.max_iter = TRANSPORT_LIN_MAX;
  a.ux = ux;
  a.uy = uy;
  a.src = c->src;
  a.s_old = s_old;
  a.s = s_new;
  hipStream_t st = c->st;
  HIPCHK(c, launch_copy(s_new, s_old, n, st));
  mrcm_transport_stats out{};
  double change = 0.0;
  int last_iters = 20;   // BiCGSTAB iterations of the previous Newton system
  for (int it = 1; it <= max_newton; ++it) {
    HIPCHK(c, launch_transport_assemble(a, st));
    // the first batch covers the previous system's iteration count and a
    // margin (successive Newton systems need similar counts); the launches
    // of a batch after convergence return at once (about 3 us each).  The
    // Newton update is queued behind every batch and applies itself only
    // once the solve has stopped, so one host read per batch sees both.
    int k = 0, batch = last_iters + 2;
    for (;;) {
      HIPCHK(c, launch_transport_bicg(a, k, batch, st));
      k += batch;
      HIPCHK(c, launch_transport_update(a, st));
      HIPCHK(c, hipMemcpyAsync(c->h_tscal, a.scal, TS_N * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipStreamSynchronize(st));
      if (c->h_tscal[TS_DONE] != 0.0 || k > a.max_iter) break;
      batch = 8;
    }
    // kernel B stops the solve at the iteration limit at the latest
    if (c->h_tscal[TS_DONE] == 0.0) return fail(c, MRCM_E_NO_CONV, "transport: BiCGSTAB did not stop");
    last_iters = std::max(4, (int)c->h_tscal[TS_ITERS]);
    out.linear_iters += (int)c->h_tscal[TS_ITERS];
    if (c->h_tscal[TS_DONE] != 1.0) out.linear_failures += 1;
    change = sqrt(c->h_tscal[TS_CHANGE]);
    out.newton_iters = it;
    if (!isfinite(change)) break;
    if (change <= eta) {
      out.converged = 1;
      break;
    }
  }
  out.last_change = change;
  out.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = out;
  if (!out.converged) {
    char msg[160];
    snprintf(msg, sizeof msg, "transport: Newton did not converge in %d iterations (last change %.3e, "
             "eta %.3e)", out.newton_iters, change, eta);
    return fail(c, MRCM_E_NO_CONV, msg);
  }
  return MRCM_OK;
}

}  // namespace

int mrcm_transport_step(mrcm_ctx* c, const double* s_old, double* s_new, const double* ux,
                        const double* uy, double dt, double s_inflow, double eta, int32_t max_newton,
                        mrcm_transport_stats* stats) {
  if (!c) return MRCM_E_INVAL;
  int r = transport_check(c, s_old, s_new, ux, uy, dt, s_inflow, eta, max_newton);
  if (r != MRCM_OK) return r;
  return transport_impl(c, s_old, s_new, ux, uy, dt, s_inflow, eta, max_newton, stats);
}

int mrcm_si_step(mrcm_ctx* c, const double* s_old, double* s_new, double* p, double* ux, double* uy,
                 double dt, double s_inflow, double eta, int32_t max_newton,
                 mrcm_transport_stats* stats) {
  if (!c) return MRCM_E_INVAL;
  int r = transport_check(c, s_old, s_new, ux, uy, dt, s_inflow, eta, max_newton);
  if (r != MRCM_OK) return r;
  if (c->precision == MRCM_PREC_SURROGATE && !c->s_ready)
    return fail(c, MRCM_E_STATE, "surrogate precision: mrcm_set_surrogate was not called");
  // s^{n+1} from u^n, then the Darcy solve with s^{n+1} (section 4)
  r = transport_impl(c, s_old, s_new, ux, uy, dt, s_inflow, eta, max_newton, stats);
  if (r != MRCM_OK) return r;
  return mrcm_step(c, s_new, 0, 1, p, ux, uy, 1, nullptr);
}

int mrcm_sfi_step(mrcm_ctx* c, const double* s_old, double* s_new, double* p, double* ux, double* uy,
                  double dt, double s_inflow, double eta, int32_t max_newton, double outer_tol,
                  int32_t max_outer, mrcm_sfi_stats* stats) {
  if (!c) return MRCM_E_INVAL;
  int r = transport_check(c, s_old, s_new, ux, uy, dt, s_inflow, eta, max_newton);
  if (r != MRCM_OK) return r;
  if (!(outer_tol > 0.0) || !isfinite(outer_tol)) return fail(c, MRCM_E_INVAL, "sfi: outer_tol must be > 0");
  if (max_outer < 1 || max_outer > 1000) return fail(c, MRCM_E_INVAL, "sfi: 1 <= max_outer <= 1000");
  if (c->precision == MRCM_PREC_SURROGATE && !c->s_ready)
    return fail(c, MRCM_E_STATE, "surrogate precision: mrcm_set_surrogate was not called");
  const auto t0 = std::chrono::steady_clock::now();
  const size_t n = (size_t)c->g.nx * c->g.ny;
  mrcm_sfi_stats out{};
  HIPCHK(c, launch_copy(s_new, s_old, n, c->st));   // s^{n+1,0} = s^n
  double change = 0.0;
  for (int k = 1; k <= max_outer; ++k) {
    // Darcy with the current iterate, then transport from s^n with its fluxes
    r = mrcm_step(c, s_new, 0, 1, p, ux, uy, 1, nullptr);
    if (r != MRCM_OK) return r;
    HIPCHK(c, launch_copy(c->s_prev, s_new, n, c->st));
    mrcm_transport_stats ts{};
    r = transport_impl(c, s_old, s_new, ux, uy, dt, s_inflow, eta, max_newton, &ts);
    out.newton_iters += ts.newton_iters;
    out.outer_iters = k;
    if (r != MRCM_OK) {
      if (stats) *stats = out;
      return r;
    }
    TransportArgs t = c->tr;
    t.nx = c->g.nx;
    t.ny = c->g.ny;
    HIPCHK(c, launch_transport_maxdiff(t, s_new, c->s_prev, c->st));
    HIPCHK(c, hipMemcpyAsync(c->h_tscal, t.scal, TS_N * sizeof(double), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    change = c->h_tscal[TS_OUTER];
    if (change < outer_tol) {
      out.converged = 1;
      break;
    }
  }
  out.last_change = change;
  out.ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (stats) *stats = out;
  if (!out.converged) {
    char msg[160];
    snprintf(msg, sizeof msg, "sfi: outer loop did not converge in %d iterations (last change %.3e)",
             out.outer_iters, change);
    return fail(c, MRCM_E_NO_CONV, msg);
  }
  return MRCM_OK;
}

const char* mrcm_last_error(const mrcm_ctx* c) {
  if (!c) return "null context";
  return c->err.c_str();
}

void mrcm_destroy(mrcm_ctx* c) {
  if (!c) return;
  if (c->st) (void)hipStreamSynchronize(c->st);
  for (void* q : c->allocs) (void)hipFree(q);
  if (c->h_report) (void)hipHostFree(c->h_report);
  if (c->h_tscal) (void)hipHostFree(c->h_tscal);
  for (hipEvent_t e : c->ev)
    if (e) (void)hipEventDestroy(e);
  if (c->own_stream && c->st) (void)hipStreamDestroy(c->st);
  delete c;
}

}  // extern "C"
