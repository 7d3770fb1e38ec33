// Vector kernels of the reduce-then-linearize interior-point method
// (Algorithm 2 of the paper). The reduced KKT system (eq. reduced:kktsystem)
// is condensed by the full-space condensation (Theorem 2): with g = 0 after
// the projection and lambda the adjoint, K_cond of the reduced system is the
// full-space one with the bounded states' slack Sigma in place of Sigma_x,
// and its right-hand side is the full-space one with r4 = 0 and the state
// rows' terms in r2. Element-wise work runs one thread per entry; the
// reductions the host reads run in one work-group (fixed summation order).
#include <hip/hip_runtime.h>

#include <cmath>

#include "redlin.hpp"

namespace rh {
namespace {

constexpr int kVec = 256;
constexpr int kRed = 1024;

__device__ __forceinline__ bool fin(double v) { return isfinite(v); }

__device__ __forceinline__ double push_in(double v, double lo, double hi, double push,
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

// Work-group reduction of kinds: 0 max, 1 min, 2 sum (blockDim = kRed).
template <int N>
__device__ void wg_reduce(double (&val)[N], const int (&kind)[N], double* out) {
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

__global__ void __launch_bounds__(kRed) k_absmax(const double* a, int n, double* out) {
  double m = 0.0;
  for (int i = threadIdx.x; i < n; i += kRed) {
    const double v = a[i];
    m = fmax(m, fin(v) ? fabs(v) : INFINITY);
  }
  double val[1] = {m};
  const int kind[1] = {0};
  wg_reduce<1>(val, kind, out);
}

__global__ void __launch_bounds__(kVec) k_fill(double* x, int n, double value) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = value;
}

__global__ void __launch_bounds__(kVec) k_redlin_adj_rhs(IpmDev v, RedLinDev R, double* b) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= v.nx) return;
  const int j = R.xbi[k];
  b[k] = -v.gl[v.nu + k] + (j >= 0 ? R.yr[R.m + j] : 0.0);
}

__global__ void __launch_bounds__(kVec) k_redlin_prep(DevNet d, IpmDev v, RedLinDev R, double mu) {
  const int nu = v.nu, nx = v.nx, nw = nu + nx, m = R.m;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nu) {
    const double lo = v.wl[i], hi = v.wu[i], x = v.w[i];
    const double il = fin(lo) ? 1.0 / (x - lo) : 0.0;
    const double iu = fin(hi) ? 1.0 / (hi - x) : 0.0;
    v.sig_w[i] = v.zl[i] * il + v.zu[i] * iu;
    v.r[i] = v.gl[i] - mu * il + mu * iu;                          // r1 = grad L_r - barrier
  }
  if (i < nx) {
    const int j = R.xbi[i];
    double sig = 0.0, r2 = 0.0;
    if (j >= 0) {
      const int q = m + j;
      const double lo = R.rsl[q], hi = R.rsu[q], s = R.sr[q];
      const double il = fin(lo) ? 1.0 / (s - lo) : 0.0;
      const double iu = fin(hi) ? 1.0 / (hi - s) : 0.0;
      sig = R.zsl[q] * il + R.zsu[q] * iu;
      const double ry = -v.w[nu + i] + s;                          // h_r + s of the state row
      const double rs = R.yr[q] - mu * il + mu * iu;
      r2 = -(sig * ry - rs);
    }
    v.sig_w[nu + i] = sig;
    v.r[i + nu] = r2;
    v.r[nw + m + i] = 0.0;                                         // r4: g = 0 (projected)
  }
  if (i < m) {
    const double lo = R.rsl[i], hi = R.rsu[i], s = R.sr[i];
    const double il = fin(lo) ? 1.0 / (s - lo) : 0.0;
    const double iu = fin(hi) ? 1.0 / (hi - s) : 0.0;
    v.sig_s[i] = R.zsl[i] * il + R.zsu[i] * iu;
    v.r[nw + i] = R.yr[i] - mu * il + mu * iu;                     // r3
    v.r[nw + m + nx + i] = d.dst[d.d_h + i] + s;                   // r5 = h + s
  }
}

__global__ void __launch_bounds__(kVec) k_redlin_pack(IpmDev v, RedLinDev R, double mu) {
  const int nu = v.nu, nx = v.nx, nw = nu + nx, m = R.m, mr = R.mr;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nu) R.rp[i] = v.p[i];
  if (i < m) {
    R.rp[nu + i] = v.p[nw + i];                                    // p_s of h
    R.rp[nu + mr + i] = v.p[nw + m + nx + i];                      // p_y of h
  }
  if (i < R.nxb) {
    const int q = m + i, k = R.xb[i];
    const double lo = R.rsl[q], hi = R.rsu[q], s = R.sr[q];
    const double il = fin(lo) ? 1.0 / (s - lo) : 0.0;
    const double iu = fin(hi) ? 1.0 / (hi - s) : 0.0;
    const double sig = R.zsl[q] * il + R.zsu[q] * iu;
    const double ps = (v.w[nu + k] - s) + v.p[nu + k];             // -(h_r + s) + S_b p_u
    R.rp[nu + q] = ps;
    R.rp[nu + mr + q] = -(R.yr[q] - mu * il + mu * iu) - sig * ps;
  }
}

__global__ void __launch_bounds__(kRed) k_dot(const double* a, const double* b, int n,
                                              double* out) {
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kRed) acc += a[i] * b[i];
  double val[1] = {acc};
  const int kind[1] = {2};
  wg_reduce<1>(val, kind, out);
}

__global__ void __launch_bounds__(kVec) k_redlin_trial_x(IpmDev v, double alpha) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < v.nx) v.wt[v.nu + k] = v.w[v.nu + k] + alpha * v.p[v.nu + k];
}

__global__ void __launch_bounds__(kRed) k_redlin_stats(DevNet d, IpmDev v, RedLinDev R,
                                                       const double* w, const double* s,
                                                       int full) {
  const int nu = v.nu, nw = nu + v.nx, m = R.m;
  const double* g = d.dst + d.d_g;
  const double* h = d.dst + d.d_h;
  double dual_w = 0.0, dual_s = 0.0, prim_g = 0.0, prim_h = 0.0;
  double dzmax = -INFINITY, dzmin = INFINITY, zsum = 0.0, lysum = 0.0, theta = 0.0;
  double logsum = 0.0, gfmax = 0.0;
  for (int i = threadIdx.x; i < nu; i += kRed) {
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
    }
  }
  if (full)
    for (int i = threadIdx.x; i < nw; i += kRed) gfmax = fmax(gfmax, fabs(v.gf[i]));
  for (int j = threadIdx.x; j < R.mr; j += kRed) {
    const double lo = R.rsl[j], hi = R.rsu[j], x = s[j];
    if (fin(lo)) {
      const double dl = x - lo;
      logsum += log(dl);
      if (full) {
        dzmax = fmax(dzmax, dl * R.zsl[j]);
        dzmin = fmin(dzmin, dl * R.zsl[j]);
      }
    }
    if (fin(hi)) {
      const double du = hi - x;
      logsum += log(du);
      if (full) {
        dzmax = fmax(dzmax, du * R.zsu[j]);
        dzmin = fmin(dzmin, du * R.zsu[j]);
      }
    }
    const double hs = (j < m ? h[j] : -w[nu + R.xb[j - m]]) + x;
    prim_h = fmax(prim_h, fabs(hs));
    theta += fabs(hs);
    if (full) {
      dual_s = fmax(dual_s, fabs(R.yr[j] - R.zsl[j] + R.zsu[j]));
      zsum += fabs(R.zsl[j]) + fabs(R.zsu[j]);
      lysum += fabs(R.yr[j]);
    }
  }
  for (int i = threadIdx.x; i < v.nx; i += kRed) prim_g = fmax(prim_g, fabs(g[i]));
  double val[11] = {dual_w, dual_s, prim_g, prim_h, dzmax, dzmin, zsum, lysum, theta, logsum,
                    gfmax};
  const int kind[11] = {0, 0, 0, 0, 0, 1, 2, 2, 2, 2, 0};
  wg_reduce<11>(val, kind, R.red);
}

__global__ void __launch_bounds__(kVec) k_redlin_init_s(DevNet d, IpmDev v, RedLinDev R,
                                                        double push, double frac) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= R.mr) return;
  const double t = j < R.m ? -d.dst[d.d_h + j] : v.w[v.nu + R.xb[j - R.m]];
  R.sr[j] = push_in(t, R.rsl[j], R.rsu[j], push, frac);
}

inline int cdiv(int a, int b) { return (a + b - 1) / b; }

}  // namespace

hipError_t launch_absmax(const double* a, int n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(k_absmax, dim3(1), dim3(kRed), 0, st, a, n, out);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, int n, double value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill, dim3(cdiv(n, kVec)), dim3(kVec), 0, st, x, n, value);
  return hipGetLastError();
}

hipError_t launch_redlin_adj_rhs(const IpmDev& v, const RedLinDev& R, double* b, hipStream_t st) {
  hipLaunchKernelGGL(k_redlin_adj_rhs, dim3(cdiv(v.nx, kVec)), dim3(kVec), 0, st, v, R, b);
  return hipGetLastError();
}

hipError_t launch_redlin_prep(const DevNet& d, const IpmDev& v, const RedLinDev& R, double mu,
                              hipStream_t st) {
  int n = v.nu > v.nx ? v.nu : v.nx;
  if (R.m > n) n = R.m;
  hipLaunchKernelGGL(k_redlin_prep, dim3(cdiv(n, kVec)), dim3(kVec), 0, st, d, v, R, mu);
  return hipGetLastError();
}

hipError_t launch_redlin_pack(const IpmDev& v, const RedLinDev& R, double mu, double* out,
                              hipStream_t st) {
  int n = v.nu > R.m ? v.nu : R.m;
  if (R.nxb > n) n = R.nxb;
  hipLaunchKernelGGL(k_redlin_pack, dim3(cdiv(n, kVec)), dim3(kVec), 0, st, v, R, mu);
  hipLaunchKernelGGL(k_dot, dim3(1), dim3(kRed), 0, st, (const double*)v.gf, (const double*)v.p,
                     v.nu + v.nx, out);
  return hipGetLastError();
}

hipError_t launch_redlin_trial_x(const IpmDev& v, double alpha, hipStream_t st) {
  hipLaunchKernelGGL(k_redlin_trial_x, dim3(cdiv(v.nx, kVec)), dim3(kVec), 0, st, v, alpha);
  return hipGetLastError();
}

hipError_t launch_redlin_stats(const DevNet& d, const IpmDev& v, const RedLinDev& R,
                               const double* w, const double* s, int full, hipStream_t st) {
  hipLaunchKernelGGL(k_redlin_stats, dim3(1), dim3(kRed), 0, st, d, v, R, w, s, full);
  return hipGetLastError();
}

hipError_t launch_redlin_init_s(const DevNet& d, const IpmDev& v, const RedLinDev& R, double push,
                                double frac, hipStream_t st) {
  hipLaunchKernelGGL(k_redlin_init_s, dim3(cdiv(R.mr > 0 ? R.mr : 1, kVec)), dim3(kVec), 0, st, d,
                     v, R, push, frac);
  return hipGetLastError();
}

}  // namespace rh
