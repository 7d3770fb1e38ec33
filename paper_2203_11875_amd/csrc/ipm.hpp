// Device vectors and kernels of the interior-point driver (Algorithm 1 of the
// paper): gradient of the Lagrangian, barrier residuals and Sigma terms,
// fraction-to-the-boundary step lengths, trial points and updates, and the
// reductions the host-side line search reads.
#pragma once

#include <hip/hip_runtime.h>

#include "device.hpp"

namespace rh {

// Reduction slots written by launch_ipm_stats / launch_ipm_dir.
enum IpmRed : int {
  IR_DUAL_W = 0,   // max |grad L - zl + zu| over w
  IR_DUAL_S = 1,   // max |y - zsl + zsu|
  IR_PRIM_G = 2,   // max |g|
  IR_PRIM_H = 3,   // max |h + s|
  IR_DZ_MAX = 4,   // max of (bound slack) * (bound multiplier) over finite bounds
  IR_DZ_MIN = 5,   // min of the same
  IR_ZSUM = 6,     // sum |z| (all bound multipliers)
  IR_LYSUM = 7,    // sum |lambda| + sum |y|
  IR_THETA = 8,    // sum |g| + sum |h + s|
  IR_LOGSUM = 9,   // sum of log(bound slack) over finite bounds (-inf if one is <= 0)
  IR_GFMAX = 10,   // max |grad f|
  IR_APRI = 11,    // largest primal step to the boundary (<= 1)
  IR_ADUAL = 12,   // largest bound-multiplier step to the boundary (<= 1)
  IR_DPHI = 13,    // directional derivative of the barrier objective
  IR_NSLOT = 16
};

// Per-instance scalars of the batched launches (kIpmSc doubles each).
enum IpmScalar : int { IS_MU = 0, IS_TAU = 1, IS_ALPHA = 2, IS_ALPHA_Z = 3, IS_ACTIVE = 4 };
constexpr int kIpmSc = 8;
enum IpmBatchOp : int { IB_LAG_GRAD, IB_STATS, IB_PREP, IB_DIR, IB_TRIAL, IB_UPDATE };

// All pointers are device memory owned by the interior-point handle; vectors
// in the library's natural order, w = [u; x].
struct IpmDev {
  int nu, nx, m;
  const double *wl, *wu, *sl, *su;    // bounds (+-inf where there is none)
  const int* u_gen;                   // nu: generator of a Pg control, else -1
  const int *gx_cptr, *gx_crow, *gx_cpos;   // G_x by internal columns: internal row, LU position
  double *w, *s, *lam, *y;
  double *zl, *zu, *zsl, *zsu;
  double *gf, *gl;                    // grad f and grad L (w order)
  double *sig_w, *sig_s;
  double *r, *p;                      // packed (r1 r2 r3 r4 r5), (p_u p_x p_s p_lambda p_y)
  double *pzl, *pzu, *pzsl, *pzsu;
  double *wt, *st;                    // trial point
  double* red;                        // IR_NSLOT doubles
  double* f;                          // [f at the iterate, f at the trial point]
};

// grad f and grad L = grad f + G^T lambda + A^T y at the point of the last
// launch_eval (derivative values in d.dst, G_x still in the LU slots).
hipError_t launch_ipm_lag_grad(const DevNet& d, const IpmDev& v, hipStream_t st);
// IR_DUAL_W .. IR_GFMAX at (w, s) (full = 0: only the primal terms, theta and
// the log-barrier sum, for a trial point).
hipError_t launch_ipm_stats(const DevNet& d, const IpmDev& v, const double* w, const double* s,
                            int full, hipStream_t st);
// Sigma_w, Sigma_s and the residuals r1..r5 of eq. kktmatrix:normal for mu.
hipError_t launch_ipm_prep(const DevNet& d, const IpmDev& v, double mu, hipStream_t st);
// bound-multiplier steps; IR_APRI, IR_ADUAL (fraction tau) and IR_DPHI.
hipError_t launch_ipm_dir(const IpmDev& v, double mu, double tau, hipStream_t st);
hipError_t launch_ipm_trial(const IpmDev& v, double alpha, hipStream_t st);
hipError_t launch_ipm_update(const IpmDev& v, double alpha, double alpha_z, double mu,
                             double kappa_sigma, hipStream_t st);
// initial point: w pushed inside its bounds, lambda = y = 0, z = 1 on finite
// bounds; then (after an evaluation at w) s = -h pushed inside its bounds.
hipError_t launch_ipm_init_w(const IpmDev& v, double push, double frac, hipStream_t st);
hipError_t launch_ipm_init_s(const DevNet& d, const IpmDev& v, double push, double frac,
                             hipStream_t st);

// One batched launch of an iteration kernel over count instances (nets,
// ipms, sc: device arrays; sc holds kIpmSc scalars per instance, instances
// with IS_ACTIVE = 0 skip). max_n: largest element count (nu + nx or m) of an
// instance for the element-wise kernels; trial / full as launch_ipm_stats
// (trial: at the trial point wt, st); ks: kappa_sigma of the update.
hipError_t launch_ipm_batch(IpmBatchOp op, const DevNet* nets, const IpmDev* ipms,
                            const double* sc, int count, int max_n, int trial, int full,
                            double ks, hipStream_t st);

// Differentiation in the loads. Outputs: pg[ng] (reference generator: -s_0),
// vm[nb], f[1] (unscaled costs); any may be null.
hipError_t launch_opf_outputs(const DevNet& d, const IpmDev& v, double inv_sigma, double* pg,
                              double* vm, double* f, hipStream_t st);
// r (packed r1..r5) = -(d outputs / d(w, s))^T (dpg, dvm, df); null weights are 0.
hipError_t launch_adjoint_rhs(const DevNet& d, const IpmDev& v, double inv_sigma,
                              const double* dpg, const double* dvm, const double* df, double* r,
                              hipStream_t st);
// gpd, gqd (nb) = -xi^T dF/d(Pd, Qd) for the packed adjoint xi (A values of the
// last evaluation in d.dst).
hipError_t launch_adjoint_grad(const DevNet& d, const IpmDev& v, const double* xi, double* gpd,
                               double* gqd, hipStream_t st);

}  // namespace rh
