// Implicit transport (transport.hip): device data, scalar slots and launch
// entry points.  Kept apart from mrcm_internal.h, which the pressure
// kernels include.
#pragma once

#include "mrcm_internal.h"

namespace mrcm {

// scalar slots (device): per iteration parity par, rho/alpha/omega of that
// iteration; shared state
enum TransportScalar {
  TS_RHO = 0,    // [2]
  TS_ALPHA = 2,  // [2]
  TS_OMEGA = 4,  // [2]
  TS_BB = 6,     // |b|^2
  TS_DONE = 7,   // 0 running, 1 converged, 2 broken down
  TS_ITERS = 8,  // iterations completed
  TS_RR = 9,     // |r|^2 at the last check
  TS_CHANGE = 10,  // Newton update: squared L2 norm of the change
  TS_OUTER = 11,   // max |a - b| of the last launch_transport_maxdiff
  TS_N = 12
};

// device data of one implicit transport step
struct TransportArgs {
  int nx, ny;
  double hx, hy, V, c;   // c = dt / V
  double M, fin;         // mu_o / mu_w; f of the injected saturation
  double tol2;           // BiCGSTAB: stop when |r|^2 <= tol2 |b|^2
  int max_iter;
  const double* ux;      // (nx+1)*ny face velocities (+x)
  const double* uy;      // nx*(ny+1) face velocities (+y)
  const double* src;     // nx*ny source per unit area, or nullptr
  const double* s_old;   // saturation at the last time level
  double* s;             // current Newton iterate
  // scaled couplings, one per face: the upwind Jacobian couples a cell only
  // to the neighbours its water comes from, so a face holds at most one
  // nonzero coupling, in the row of its downstream cell; all couplings are
  // <= 0.  cfx ((nx+1)*ny x-faces, face (i, j) west of cell (i, j)) holds
  // the east cell's coupling to the west cell when the flow is +x, minus
  // the west cell's coupling to the east cell when it is -x; cfy
  // (nx*(ny+1) y-faces) likewise with south and north.  A cell's couplings
  // are min(west face, 0), -max(east face, 0), min(south face, 0) and
  // -max(north face, 0).
  double* cfx; double* cfy;
  double* x;             // Newton direction (BiCGSTAB solution)
  double* r; double* rh; double* p[2]; double* v[2]; double* q; double* t;
  double* part[3];       // per-work-group partial sums (up to 4 per work-group)
  double* scal;          // TS_* slots
};

int transport_blocks(int nx, int ny);   // work-groups of a cell-wise launch (partials per kernel)
// residual and scaled Jacobian at the current iterate, BiCGSTAB start
hipError_t launch_transport_assemble(const TransportArgs& a, hipStream_t st);
// BiCGSTAB iterations k0 .. k0+count-1 (launches after convergence return at once)
hipError_t launch_transport_bicg(const TransportArgs& a, int k0, int count, hipStream_t st);
// Newton update (bound, inflection-point rule) and the squared norm of the
// change; does nothing while scal[TS_DONE] is 0 (the solve has not stopped)
hipError_t launch_transport_update(const TransportArgs& a, hipStream_t st);
// max |a - b| over the cells into scal[TS_OUTER]
hipError_t launch_transport_maxdiff(const TransportArgs& t, const double* a, const double* b,
                                   hipStream_t st);

}  // namespace mrcm
