// Vector kernels of the reduce-then-linearize interior-point method
// (Algorithm 2 of the paper): power-flow residual checks for the projection,
// the adjoint right-hand side, Sigma and residuals of the reduced KKT system
// mapped onto the full-space condensation, the reduced step, and the
// reductions the host-side line search reads.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"
#include "ipm.hpp"

namespace rh {

// Reduced-space variables: the slack and multiplier vectors of
// h_r = [h; -x_b] (m + nxb entries: the m rows of h, then the bounded states
// x_b = x[xb[j]]), their bounds, bound multipliers and step. Device memory
// owned by the RedLin handle; x, u, lambda, y_h live in the full-space
// IpmDev (w = [u; x], y = the first m entries of yr).
struct RedLinDev {
  int m, mr, nxb;
  const int* xb;           // nxb: natural x index of each bounded state
  const int* xbi;          // nx: position in xb, or -1
  const double *rsl, *rsu; // mr: bounds of the slacks (+-inf where none)
  double *sr, *yr;         // mr: slacks s_r, multipliers y_r
  double *zsl, *zsu;       // mr: slack bound multipliers
  double* rp;              // nu + 2 mr: reduced step (p_u, p_s, p_y)
  double *pzsl, *pzsu;     // mr
  double* st;              // mr: trial slacks
  double* zero;            // nu zeros (reduced objective gradient placeholder)
  double* red;             // IR_NSLOT doubles
};

// out[0] = max |a_i| over n entries (+inf if one is not finite).
hipError_t launch_absmax(const double* a, int n, double* out, hipStream_t st);
// b = -(grad_x f + A_x^T y_h - y_x) from gl computed with lambda = 0 (natural x).
hipError_t launch_redlin_adj_rhs(const IpmDev& v, const RedLinDev& R, double* b, hipStream_t st);
// Sigma_u, Sigma of the bounded states (as Sigma_x), Sigma_s of h and the
// full-space residuals r1..r5 whose condensation is the reduced system's.
hipError_t launch_redlin_prep(const DevNet& d, const IpmDev& v, const RedLinDev& R, double mu,
                              hipStream_t st);
// The reduced step (p_u, p_s, p_y) from the full-space step in v.p, and
// out[0] = grad f . (p_u, p_x) (the objective part of the directional derivative).
hipError_t launch_redlin_pack(const IpmDev& v, const RedLinDev& R, double mu, double* out,
                              hipStream_t st);
// trial state warm start: wt_x = x + alpha p_x.
hipError_t launch_redlin_trial_x(const IpmDev& v, double alpha, hipStream_t st);
// reductions at (w, s_r) into R.red (IpmRed slots; full = 0: primal terms only).
hipError_t launch_redlin_stats(const DevNet& d, const IpmDev& v, const RedLinDev& R,
                               const double* w, const double* s, int full, hipStream_t st);
// initial slacks: s_r = [-h; x_b] pushed inside their bounds.
hipError_t launch_redlin_init_s(const DevNet& d, const IpmDev& v, const RedLinDev& R, double push,
                                double frac, hipStream_t st);
hipError_t launch_fill(double* x, int n, double value, hipStream_t st);

}  // namespace rh
