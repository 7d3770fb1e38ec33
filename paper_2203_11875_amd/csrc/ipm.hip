// Vector kernels of the interior-point driver (Algorithm 1 of the paper with a
// filter line search). Element-wise work runs one thread per entry; every
// reduction the host reads runs in one work-group so that its summation
// order is fixed (repeatable runs).
#include <hip/hip_runtime.h>

#include <cmath>

#include "ipm.hpp"

namespace rh {
namespace {

constexpr int kVec = 256;
constexpr int kRed = 1024;

__device__ __forceinline__ bool fin(double v) { return isfinite(v); }

// Moves v strictly inside [lo, hi] (finite sides only): by
// push * max(1, |bound|), at most frac of the width when both sides exist.
__device__ __forceinline__ double push_inside(double v, double lo, double hi, double push,
                                              double frac) {
  const bool fl = fin(lo), fu = fin(hi);
  double pl = fl ? push * fmax(1.0, fabs(lo)) : 0.0;
  double pu = fu ? push * fmax(1.0, fabs(hi)) : 0.0;
  if (fl && fu) {
    pl = fmin(pl, frac * (hi - lo));
    pu = fmin(pu, frac * (hi - lo));
  }
  if (fl) v = fmax(v, lo + pl);
  if (fu) v = fmin(v, hi - pu);
  return v;
}

__device__ __forceinline__ void ipm_lag_grad_body(const DevNet& d, const IpmDev& v) {
  const int nw = v.nu + v.nx;
  const int vi = blockIdx.x * blockDim.x + threadIdx.x;
  if (vi >= nw) return;
  const double* A = d.dst + d.d_a;
  const double B = d.base;
  // Pg_ref = h_0 is a function of the state: its cost derivative multiplies
  // the first row of A (the gradient of h_0)
  const double fref = B * (2.0 * d.c2_ref * B * d.dst[d.d_h] + d.c1_ref);
  double gfv = 0.0, acc = 0.0;
  int out;
  if (vi < v.nu) {
    out = vi;
    const int g = v.u_gen[vi];
    if (g >= 0) gfv = B * (2.0 * d.c2[g] * B * v.w[vi] + d.c1[g]);
    const double* Gu = d.dst + d.d_gu;
    for (int e = d.gucsc_ptr[vi]; e < d.gucsc_ptr[vi + 1]; ++e)
      acc += Gu[d.gucsc_from[e]] * v.lam[d.perm[d.gucsc_row[e]]];
  } else {
    const int ci = vi - v.nu;
    out = v.nu + d.perm[ci];
    const double* LU = d.dst + d.d_lu;
    for (int e = v.gx_cptr[ci]; e < v.gx_cptr[ci + 1]; ++e)
      acc += LU[v.gx_cpos[e]] * v.lam[d.perm[v.gx_crow[e]]];
  }
  for (int e = d.acsc_ptr[vi]; e < d.acsc_ptr[vi + 1]; ++e) {
    const int j = d.acsc_row[e];
    const double a = A[d.acsc_from[e]];
    acc += a * v.y[j];
    if (j == 0) gfv += fref * a;
  }
  v.gf[out] = gfv;
  v.gl[out] = gfv + acc;
}
__global__ void __launch_bounds__(kVec) k_ipm_lag_grad(DevNet d, IpmDev v) {
  ipm_lag_grad_body(d, v);
}

// Work-group reduction of kinds: 0 max, 1 min, 2 sum.
template <int N>
__device__ void block_reduce(double (&val)[N], const int (&kind)[N], double* out) {
  __shared__ double buf[N][kRed / 64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < N; ++q) {
    double x = val[q];
    for (int off = 32; off > 0; off >>= 1) {
      const double o = __shfl_xor(x, off);
      x = kind[q] == 0 ? fmax(x, o) : kind[q] == 1 ? fmin(x, o) : x + o;
    }
    if (lane == 0) buf[q][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x < N) {
    const int q = threadIdx.x;
    double x = buf[q][0];
    for (int k = 1; k < kRed / 64; ++k)
      x = kind[q] == 0 ? fmax(x, buf[q][k]) : kind[q] == 1 ? fmin(x, buf[q][k]) : x + buf[q][k];
    out[q] = x;
  }
}

__device__ __forceinline__ void ipm_stats_body(const DevNet& d, const IpmDev& v, const double* w,
                                               const double* s, int full) {
  const int nw = v.nu + v.nx;
  const double* g = d.dst + d.d_g;
  const double* h = d.dst + d.d_h;
  double dual_w = 0.0, dual_s = 0.0, prim_g = 0.0, prim_h = 0.0;
  double dzmax = -INFINITY, dzmin = INFINITY, zsum = 0.0, lysum = 0.0, theta = 0.0;
  double logsum = 0.0, gfmax = 0.0;
  for (int i = threadIdx.x; i < nw; i += kRed) {
    const double lo = v.wl[i], hi = v.wu[i], x = w[i];
    if (fin(lo)) {
      const double dl = x - lo;
      logsum += log(dl);
      if (full) {
        dzmax = fmax(dzmax, dl * v.zl[i]);
        dzmin = fmin(dzmin, dl * v.zl[i]);
      }
    }
    if (fin(hi)) {
      const double du = hi - x;
      logsum += log(du);
      if (full) {
        dzmax = fmax(dzmax, du * v.zu[i]);
        dzmin = fmin(dzmin, du * v.zu[i]);
      }
    }
    if (full) {
      dual_w = fmax(dual_w, fabs(v.gl[i] - v.zl[i] + v.zu[i]));
      zsum += fabs(v.zl[i]) + fabs(v.zu[i]);
      gfmax = fmax(gfmax, fabs(v.gf[i]));
    }
  }
  for (int j = threadIdx.x; j < v.m; j += kRed) {
    const double lo = v.sl[j], hi = v.su[j], x = s[j];
    if (fin(lo)) {
      const double dl = x - lo;
      logsum += log(dl);
      if (full) {
        dzmax = fmax(dzmax, dl * v.zsl[j]);
        dzmin = fmin(dzmin, dl * v.zsl[j]);
      }
    }
    if (fin(hi)) {
      const double du = hi - x;
      logsum += log(du);
      if (full) {
        dzmax = fmax(dzmax, du * v.zsu[j]);
        dzmin = fmin(dzmin, du * v.zsu[j]);
      }
    }
    const double hs = h[j] + x;
    prim_h = fmax(prim_h, fabs(hs));
    theta += fabs(hs);
    if (full) {
      dual_s = fmax(dual_s, fabs(v.y[j] - v.zsl[j] + v.zsu[j]));
      zsum += fabs(v.zsl[j]) + fabs(v.zsu[j]);
      lysum += fabs(v.y[j]);
    }
  }
  for (int i = threadIdx.x; i < v.nx; i += kRed) {
    prim_g = fmax(prim_g, fabs(g[i]));
    theta += fabs(g[i]);
    if (full) lysum += fabs(v.lam[i]);
  }
  double val[11] = {dual_w, dual_s, prim_g, prim_h, dzmax, dzmin, zsum, lysum, theta, logsum,
                    gfmax};
  const int kind[11] = {0, 0, 0, 0, 0, 1, 2, 2, 2, 2, 0};
  block_reduce<11>(val, kind, v.red);
}
__global__ void __launch_bounds__(kRed) k_ipm_stats(DevNet d, IpmDev v, const double* w, const double* s, int full) {
  ipm_stats_body(d, v, w, s, full);
}

__device__ __forceinline__ void ipm_prep_body(const DevNet& d, const IpmDev& v, double mu) {
  const int nw = v.nu + v.nx;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) {
    const double lo = v.wl[i], hi = v.wu[i], x = v.w[i];
    const double il = fin(lo) ? 1.0 / (x - lo) : 0.0;
    const double iu = fin(hi) ? 1.0 / (hi - x) : 0.0;
    v.sig_w[i] = v.zl[i] * il + v.zu[i] * iu;
    v.r[i] = v.gl[i] - mu * il + mu * iu;                 // r1 (u), r2 (x)
  }
  if (i < v.m) {
    const double lo = v.sl[i], hi = v.su[i], x = v.s[i];
    const double il = fin(lo) ? 1.0 / (x - lo) : 0.0;
    const double iu = fin(hi) ? 1.0 / (hi - x) : 0.0;
    v.sig_s[i] = v.zsl[i] * il + v.zsu[i] * iu;
    v.r[nw + i] = v.y[i] - mu * il + mu * iu;             // r3
    v.r[nw + v.m + v.nx + i] = d.dst[d.d_h + i] + x;      // r5 = h + s
  }
  if (i < v.nx) v.r[nw + v.m + i] = d.dst[d.d_g + i];     // r4 = g
}
__global__ void __launch_bounds__(kVec) k_ipm_prep(DevNet d, IpmDev v, double mu) {
  ipm_prep_body(d, v, mu);
}

__device__ __forceinline__ void ipm_dir_body(const IpmDev& v, double mu, double tau) {
  const int nw = v.nu + v.nx;
  double apri = 1.0, adual = 1.0, dphi = 0.0;
  for (int i = threadIdx.x; i < nw; i += kRed) {
    const double pw = v.p[i], lo = v.wl[i], hi = v.wu[i], x = v.w[i];
    double pzl = 0.0, pzu = 0.0;
    if (fin(lo)) {
      const double dl = x - lo, il = 1.0 / dl;
      pzl = mu * il - v.zl[i] - v.zl[i] * il * pw;
      if (pw < 0.0) apri = fmin(apri, -tau * dl / pw);
      if (pzl < 0.0) adual = fmin(adual, -tau * v.zl[i] / pzl);
      dphi -= mu * il * pw;
    }
    if (fin(hi)) {
      const double du = hi - x, iu = 1.0 / du;
      pzu = mu * iu - v.zu[i] + v.zu[i] * iu * pw;
      if (pw > 0.0) apri = fmin(apri, tau * du / pw);
      if (pzu < 0.0) adual = fmin(adual, -tau * v.zu[i] / pzu);
      dphi += mu * iu * pw;
    }
    v.pzl[i] = pzl;
    v.pzu[i] = pzu;
    dphi += v.gf[i] * pw;
  }
  for (int j = threadIdx.x; j < v.m; j += kRed) {
    const double ps = v.p[nw + j], lo = v.sl[j], hi = v.su[j], x = v.s[j];
    double pzl = 0.0, pzu = 0.0;
    if (fin(lo)) {
      const double dl = x - lo, il = 1.0 / dl;
      pzl = mu * il - v.zsl[j] - v.zsl[j] * il * ps;
      if (ps < 0.0) apri = fmin(apri, -tau * dl / ps);
      if (pzl < 0.0) adual = fmin(adual, -tau * v.zsl[j] / pzl);
      dphi -= mu * il * ps;
    }
    if (fin(hi)) {
      const double du = hi - x, iu = 1.0 / du;
      pzu = mu * iu - v.zsu[j] + v.zsu[j] * iu * ps;
      if (ps > 0.0) apri = fmin(apri, tau * du / ps);
      if (pzu < 0.0) adual = fmin(adual, -tau * v.zsu[j] / pzu);
      dphi += mu * iu * ps;
    }
    v.pzsl[j] = pzl;
    v.pzsu[j] = pzu;
  }
  double val[3] = {apri, adual, dphi};
  const int kind[3] = {1, 1, 2};
  block_reduce<3>(val, kind, v.red + IR_APRI);
}
__global__ void __launch_bounds__(kRed) k_ipm_dir(IpmDev v, double mu, double tau) {
  ipm_dir_body(v, mu, tau);
}

__device__ __forceinline__ void ipm_trial_body(const IpmDev& v, double alpha) {
  const int nw = v.nu + v.nx;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) v.wt[i] = v.w[i] + alpha * v.p[i];
  if (i < v.m) v.st[i] = v.s[i] + alpha * v.p[nw + i];
}
__global__ void __launch_bounds__(kVec) k_ipm_trial(IpmDev v, double alpha) {
  ipm_trial_body(v, alpha);
}

__device__ __forceinline__ double clip_z(double z, double d, double mu, double k) {
  return fmin(fmax(z, mu / (k * d)), k * mu / d);
}

__device__ __forceinline__ void ipm_update_body(const IpmDev& v, double alpha, double alpha_z,
                                                double mu, double ks) {
  const int nw = v.nu + v.nx;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) {
    const double x = v.w[i] + alpha * v.p[i];
    v.w[i] = x;
    const double lo = v.wl[i], hi = v.wu[i];
    v.zl[i] = fin(lo) ? clip_z(v.zl[i] + alpha_z * v.pzl[i], x - lo, mu, ks) : 0.0;
    v.zu[i] = fin(hi) ? clip_z(v.zu[i] + alpha_z * v.pzu[i], hi - x, mu, ks) : 0.0;
  }
  if (i < v.m) {
    const double x = v.s[i] + alpha * v.p[nw + i];
    v.s[i] = x;
    const double lo = v.sl[i], hi = v.su[i];
    v.zsl[i] = fin(lo) ? clip_z(v.zsl[i] + alpha_z * v.pzsl[i], x - lo, mu, ks) : 0.0;
    v.zsu[i] = fin(hi) ? clip_z(v.zsu[i] + alpha_z * v.pzsu[i], hi - x, mu, ks) : 0.0;
    v.y[i] += alpha * v.p[nw + v.m + v.nx + i];
  }
  if (i < v.nx) v.lam[i] += alpha * v.p[nw + v.m + i];
}
__global__ void __launch_bounds__(kVec) k_ipm_update(IpmDev v, double alpha, double alpha_z, double mu, double ks) {
  ipm_update_body(v, alpha, alpha_z, mu, ks);
}

__global__ void __launch_bounds__(kVec) k_ipm_init_w(IpmDev v, double push, double frac) {
  const int nw = v.nu + v.nx;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nw) {
    v.w[i] = push_inside(v.w[i], v.wl[i], v.wu[i], push, frac);
    v.zl[i] = fin(v.wl[i]) ? 1.0 : 0.0;
    v.zu[i] = fin(v.wu[i]) ? 1.0 : 0.0;
  }
  if (i < v.m) {
    v.zsl[i] = fin(v.sl[i]) ? 1.0 : 0.0;
    v.zsu[i] = fin(v.su[i]) ? 1.0 : 0.0;
    v.y[i] = 0.0;
  }
  if (i < v.nx) v.lam[i] = 0.0;
}

__global__ void __launch_bounds__(kVec) k_ipm_init_s(DevNet d, IpmDev v, double push,
                                                    double frac) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < v.m) v.s[j] = push_inside(-d.dst[d.d_h + j], v.sl[j], v.su[j], push, frac);
}

// ---------------------------------------------------------------------------
// Differentiation of the solution in the loads (implicit function theorem at
// the final barrier problem; the adjoint system is K_aug, symmetric, solved
// through the same condensation).

// Outputs: Pg of every generator (the reference generator's is -s_0, which
// equals h_0 at a solution), Vm of every bus, f with unscaled costs.
__global__ void __launch_bounds__(kRed) k_opf_outputs(DevNet d, IpmDev v, double inv_sigma,
                                                     double* pg, double* vm, double* f) {
  if (vm)
    for (int i = threadIdx.x; i < d.nb; i += kRed)
      vm[i] = d.vmu[i] >= 0 ? v.w[d.vmu[i]] : v.w[v.nu + d.vmx_nat[i]];
  double acc = 0.0;
  for (int g = threadIdx.x; g < d.ng; g += kRed) {
    const double p = d.pg_u[g] >= 0 ? v.w[d.pg_u[g]] : -v.s[0];
    if (pg) pg[g] = p;
    const double bp = d.base * p;
    acc += (d.c2[g] * bp * bp + d.c1[g] * bp + d.c0[g]) * inv_sigma;
  }
  __shared__ double res[1];
  double val[1] = {acc};
  const int kind[1] = {2};
  block_reduce<1>(val, kind, res);
  __syncthreads();
  if (threadIdx.x == 0 && f) f[0] = res[0];
}

__global__ void __launch_bounds__(kVec) k_fill_zero(double* x, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = 0.0;
}

// r = -c with c = (d outputs / d(w, s))^T (dpg, dvm, df); zero elsewhere
// (cleared before). The Vm and Pg entries of u and the Vm entries of x are
// distinct, so every thread writes its own entry.
__global__ void __launch_bounds__(kVec) k_adjoint_rhs(DevNet d, IpmDev v, double inv_sigma,
                                                     const double* dpg, const double* dvm,
                                                     const double* df, double* r) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t < d.nb && dvm) r[d.vmu[t] >= 0 ? d.vmu[t] : v.nu + d.vmx_nat[t]] = -dvm[t];
  if (t < d.ng) {
    const int k = d.pg_u[t];
    const double p = k >= 0 ? v.w[k] : -v.s[0];
    const double dcost = d.base * (2.0 * d.c2[t] * d.base * p + d.c1[t]) * inv_sigma;
    const double c = (dpg ? dpg[t] : 0.0) + (df ? df[0] * dcost : 0.0);
    if (k >= 0) r[k] = -c;
    else r[v.nu + v.nx] = c;            // Pg_ref = -s_0: c_s0 = -c
  }
}

// grad_p = -xi^T dF/dp: the loads enter the P and Q balance rows (lambda),
// h_0 = Pg_ref and h_{1+g} = Qg (y), and through the cost of Pg_ref the
// stationarity rows, as 2 c2_ref base^2 (grad h_0) in Pd_ref.
__global__ void __launch_bounds__(kRed) k_adjoint_grad(DevNet d, IpmDev v, const double* xi,
                                                      double* gpd, double* gqd) {
  const int nw = v.nu + v.nx;
  const double* xl = xi + nw + v.m;
  const double* xy = xl + v.nx;
  const double* A = d.dst + d.d_a;
  double acc = 0.0;
  for (int e = d.a_ptr[0] + threadIdx.x; e < d.a_ptr[1]; e += kRed) {
    const int c = d.a_col[e];
    acc += A[e] * xi[c < v.nu ? c : v.nu + d.perm[c - v.nu]];
  }
  __shared__ double a0[1];
  double val[1] = {acc};
  const int kind[1] = {2};
  block_reduce<1>(val, kind, a0);
  __syncthreads();
  const double cref = 2.0 * d.c2_ref * d.base * d.base * a0[0];
  for (int i = threadIdx.x; i < d.nb; i += kRed) {
    double gp = d.th_nat[i] >= 0 ? xl[d.th_nat[i]] : 0.0;
    if (i == d.ref) gp += xy[0] + cref;
    double gq = d.vmx_nat[i] >= 0 ? xl[d.vmx_nat[i]] : 0.0;
    if (d.vmu[i] >= 0) gq += xy[1 + d.vmu[i]];
    gpd[i] = -gp;
    gqd[i] = -gq;
  }
}

// ---------------------------------------------------------------------------
// Batched forms (instance = blockIdx.z) for solvers stepped in lockstep: the
// same bodies, per-instance scalars in sc (IpmScalar slots), instances whose
// active slot is 0 skip the launch.
__device__ __forceinline__ bool ipm_active(const double* sc) {
  return sc[kIpmSc * blockIdx.z + IS_ACTIVE] != 0.0;
}
__global__ void __launch_bounds__(kVec) k_ipm_lag_grad_b(const DevNet* nets, const IpmDev* ipms,
                                                        const double* sc) {
  if (!ipm_active(sc)) return;
  ipm_lag_grad_body(cst(nets, blockIdx.z), cst(ipms, blockIdx.z));
}
__global__ void __launch_bounds__(kRed) k_ipm_stats_b(const DevNet* nets, const IpmDev* ipms,
                                                     const double* sc, int trial, int full) {
  if (!ipm_active(sc)) return;
  const IpmDev& v = cst(ipms, blockIdx.z);
  ipm_stats_body(cst(nets, blockIdx.z), v, trial ? v.wt : v.w, trial ? v.st : v.s, full);
}
__global__ void __launch_bounds__(kVec) k_ipm_prep_b(const DevNet* nets, const IpmDev* ipms,
                                                    const double* sc) {
  if (!ipm_active(sc)) return;
  ipm_prep_body(cst(nets, blockIdx.z), cst(ipms, blockIdx.z), sc[kIpmSc * blockIdx.z + IS_MU]);
}
__global__ void __launch_bounds__(kRed) k_ipm_dir_b(const IpmDev* ipms, const double* sc) {
  if (!ipm_active(sc)) return;
  const double* q = sc + kIpmSc * blockIdx.z;
  ipm_dir_body(cst(ipms, blockIdx.z), q[IS_MU], q[IS_TAU]);
}
__global__ void __launch_bounds__(kVec) k_ipm_trial_b(const IpmDev* ipms, const double* sc) {
  if (!ipm_active(sc)) return;
  ipm_trial_body(cst(ipms, blockIdx.z), sc[kIpmSc * blockIdx.z + IS_ALPHA]);
}
__global__ void __launch_bounds__(kVec) k_ipm_update_b(const IpmDev* ipms, const double* sc,
                                                      double ks) {
  if (!ipm_active(sc)) return;
  const double* q = sc + kIpmSc * blockIdx.z;
  ipm_update_body(cst(ipms, blockIdx.z), q[IS_ALPHA], q[IS_ALPHA_Z], q[IS_MU], ks);
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }
inline int vec_grid(const IpmDev& v) {
  int n = v.nu + v.nx;
  if (v.m > n) n = v.m;
  return cdiv(n > 0 ? n : 1, kVec);
}

}  // namespace

hipError_t launch_ipm_lag_grad(const DevNet& d, const IpmDev& v, hipStream_t st) {
  hipLaunchKernelGGL(k_ipm_lag_grad, dim3(cdiv(v.nu + v.nx, kVec)), dim3(kVec), 0, st, d, v);
  return hipGetLastError();
}

hipError_t launch_ipm_stats(const DevNet& d, const IpmDev& v, const double* w, const double* s,
                            int full, hipStream_t st) {
  hipLaunchKernelGGL(k_ipm_stats, dim3(1), dim3(kRed), 0, st, d, v, w, s, full);
  return hipGetLastError();
}

hipError_t launch_ipm_prep(const DevNet& d, const IpmDev& v, double mu, hipStream_t st) {
  hipLaunchKernelGGL(k_ipm_prep, dim3(vec_grid(v)), dim3(kVec), 0, st, d, v, mu);
  return hipGetLastError();
}

hipError_t launch_ipm_dir(const IpmDev& v, double mu, double tau, hipStream_t st) {
  hipLaunchKernelGGL(k_ipm_dir, dim3(1), dim3(kRed), 0, st, v, mu, tau);
  return hipGetLastError();
}

hipError_t launch_ipm_trial(const IpmDev& v, double alpha, hipStream_t st) {
  hipLaunchKernelGGL(k_ipm_trial, dim3(vec_grid(v)), dim3(kVec), 0, st, v, alpha);
  return hipGetLastError();
}

hipError_t launch_ipm_update(const IpmDev& v, double alpha, double alpha_z, double mu,
                             double kappa_sigma, hipStream_t st) {
  hipLaunchKernelGGL(k_ipm_update, dim3(vec_grid(v)), dim3(kVec), 0, st, v, alpha, alpha_z, mu,
                     kappa_sigma);
  return hipGetLastError();
}

hipError_t launch_ipm_init_w(const IpmDev& v, double push, double frac, hipStream_t st) {
  hipLaunchKernelGGL(k_ipm_init_w, dim3(vec_grid(v)), dim3(kVec), 0, st, v, push, frac);
  return hipGetLastError();
}

hipError_t launch_ipm_init_s(const DevNet& d, const IpmDev& v, double push, double frac,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_ipm_init_s, dim3(cdiv(v.m > 0 ? v.m : 1, kVec)), dim3(kVec), 0, st, d, v,
                     push, frac);
  return hipGetLastError();
}

hipError_t launch_opf_outputs(const DevNet& d, const IpmDev& v, double inv_sigma, double* pg,
                              double* vm, double* f, hipStream_t st) {
  hipLaunchKernelGGL(k_opf_outputs, dim3(1), dim3(kRed), 0, st, d, v, inv_sigma, pg, vm, f);
  return hipGetLastError();
}

hipError_t launch_adjoint_rhs(const DevNet& d, const IpmDev& v, double inv_sigma,
                              const double* dpg, const double* dvm, const double* df, double* r,
                              hipStream_t st) {
  const int np = v.nu + 2 * v.nx + 2 * v.m;
  hipLaunchKernelGGL(k_fill_zero, dim3(cdiv(np, kVec)), dim3(kVec), 0, st, r, np);
  const int n = d.nb > d.ng ? d.nb : d.ng;
  hipLaunchKernelGGL(k_adjoint_rhs, dim3(cdiv(n, kVec)), dim3(kVec), 0, st, d, v, inv_sigma, dpg,
                     dvm, df, r);
  return hipGetLastError();
}

hipError_t launch_adjoint_grad(const DevNet& d, const IpmDev& v, const double* xi, double* gpd,
                               double* gqd, hipStream_t st) {
  hipLaunchKernelGGL(k_adjoint_grad, dim3(1), dim3(kRed), 0, st, d, v, xi, gpd, gqd);
  return hipGetLastError();
}

hipError_t launch_ipm_batch(IpmBatchOp op, const DevNet* nets, const IpmDev* ipms,
                            const double* sc, int count, int max_n, int trial, int full,
                            double ks, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const dim3 vg(cdiv(max_n > 0 ? max_n : 1, kVec), 1, count), rg(1, 1, count);
  switch (op) {
    case IB_LAG_GRAD:
      hipLaunchKernelGGL(k_ipm_lag_grad_b, vg, dim3(kVec), 0, st, nets, ipms, sc);
      break;
    case IB_STATS:
      hipLaunchKernelGGL(k_ipm_stats_b, rg, dim3(kRed), 0, st, nets, ipms, sc, trial, full);
      break;
    case IB_PREP:
      hipLaunchKernelGGL(k_ipm_prep_b, vg, dim3(kVec), 0, st, nets, ipms, sc);
      break;
    case IB_DIR:
      hipLaunchKernelGGL(k_ipm_dir_b, rg, dim3(kRed), 0, st, ipms, sc);
      break;
    case IB_TRIAL:
      hipLaunchKernelGGL(k_ipm_trial_b, vg, dim3(kVec), 0, st, ipms, sc);
      break;
    case IB_UPDATE:
      hipLaunchKernelGGL(k_ipm_update_b, vg, dim3(kVec), 0, st, ipms, sc, ks);
      break;
  }
  return hipGetLastError();
}

}  // namespace rh
