// HIP kernels (gfx950) of the condensation hot path:
//   derivative values on fixed patterns, static-pivot refactorisation of G_x,
//   the fused tangent-solve / Hessian-product / adjoint-solve pipeline that
//   builds K_cond column blocks, symmetrisation, blocked Cholesky with the
//   forward substitution folded into the panel step, backward substitution,
//   and the step recovery.
#include <hip/hip_runtime.h>

#include <cmath>

#include "analysis.hpp"
#include "device.hpp"

namespace rh {

namespace {

constexpr int kBlock = 256;

__device__ inline double bus_theta(const DevNet& d, const double* x, int i) {
  int k = d.th_nat[i];
  return k >= 0 ? x[k] : 0.0;
}
__device__ inline double bus_vm(const DevNet& d, const double* x, const double* u, int i) {
  int k = d.vmx_nat[i];
  return k >= 0 ? x[k] : u[d.vmu[i]];
}

// F = alpha * Va^2 + Vf Vt kap(phi), phi = theta_f - theta_t, kap'' = -kap,
// with Va the voltage at the end the function belongs to. Local variables
// (theta_f, theta_t, Vf, Vt); Hessian as 10 upper-triangle entries.
__device__ inline void line_fun(double alpha, double kap, double kapd, double vf, double vt,
                                bool at_from, double* val, double* g, double* H) {
  const double V = vf * vt;
  const double va = at_from ? vf : vt;
  *val = alpha * va * va + V * kap;
  g[0] = V * kapd;
  g[1] = -V * kapd;
  g[2] = vt * kap + (at_from ? 2.0 * alpha * vf : 0.0);
  g[3] = vf * kap + (at_from ? 0.0 : 2.0 * alpha * vt);
  H[0] = -V * kap;        // (th_f, th_f)
  H[1] = V * kap;         // (th_f, th_t)
  H[2] = vt * kapd;       // (th_f, V_f)
  H[3] = vf * kapd;       // (th_f, V_t)
  H[4] = -V * kap;        // (th_t, th_t)
  H[5] = -vt * kapd;      // (th_t, V_f)
  H[6] = -vf * kapd;      // (th_t, V_t)
  H[7] = at_from ? 2.0 * alpha : 0.0;   // (V_f, V_f)
  H[8] = kap;             // (V_f, V_t)
  H[9] = at_from ? 0.0 : 2.0 * alpha;   // (V_t, V_t)
}

struct LineTrig {
  double vf, vt, a, b, e, q;
};

__device__ inline LineTrig line_trig(const DevNet& d, const double* x, const double* u, int l) {
  const int f = d.lf[l], t = d.lt[l];
  double s, c;
  sincos(bus_theta(d, x, f) - bus_theta(d, x, t), &s, &c);
  const double G = d.gft[l], B = d.bft[l];
  LineTrig r;
  r.vf = bus_vm(d, x, u, f);
  r.vt = bus_vm(d, x, u, t);
  r.a = G * c + B * s;    // P_from mutual term  (derivative -b)
  r.b = G * s - B * c;    // Q_from mutual term  (derivative  a)
  r.e = G * c - B * s;    // P_to mutual term    (derivative  q)
  r.q = -G * s - B * c;   // Q_to mutual term    (derivative -e)
  return r;
}

__device__ double ref_injection(const DevNet& d, const double* x, const double* u) {
  double p = 0.0;
  for (int k = 0; k < d.n_ref_lines; ++k) {
    const int l = d.ref_lines[k];
    const LineTrig tr = line_trig(d, x, u, l);
    if (d.ref_ends[k] == 0)
      p += d.gff[l] * tr.vf * tr.vf + tr.vf * tr.vt * tr.a;
    else
      p += d.gff[l] * tr.vt * tr.vt + tr.vf * tr.vt * tr.e;
  }
  return p;
}

// ---------------------------------------------------------------- evaluation
__global__ void __launch_bounds__(kBlock) k_eval_lines(DevNet d, const double* x, const double* u,
                                                      const double* lam, const double* y,
                                                      int hessian) {
  const int l = blockIdx.x * blockDim.x + threadIdx.x;
  if (l < d.nu) d.src[d.src_u + l] = u[l];
  if (l >= d.nl) return;
  const LineTrig tr = line_trig(d, x, u, l);
  const double gff = d.gff[l], bff = d.bff[l];
  double Pf, Qf, Pt, Qt, gPf[4], gQf[4], gPt[4], gQt[4], HPf[10], HQf[10], HPt[10], HQt[10];
  line_fun(gff, tr.a, -tr.b, tr.vf, tr.vt, true, &Pf, gPf, HPf);
  line_fun(-bff, tr.b, tr.a, tr.vf, tr.vt, true, &Qf, gQf, HQf);
  line_fun(gff, tr.e, tr.q, tr.vf, tr.vt, false, &Pt, gPt, HPt);
  line_fun(-bff, tr.q, -tr.e, tr.vf, tr.vt, false, &Qt, gQt, HQt);
  double* o = d.src + (size_t)LF_STRIDE * l;
  o[LF_PF] = Pf;
  o[LF_QF] = Qf;
  o[LF_PT] = Pt;
  o[LF_QT] = Qt;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o[LF_DPF + k] = gPf[k];
    o[LF_DQF + k] = gQf[k];
    o[LF_DPT + k] = gPt[k];
    o[LF_DQT + k] = gQt[k];
    o[LF_DSF2 + k] = 2.0 * (Pf * gPf[k] + Qf * gQf[k]);
    o[LF_DST2 + k] = 2.0 * (Pt * gPt[k] + Qt * gQt[k]);
  }
  o[LF_SF2] = Pf * Pf + Qf * Qf;
  o[LF_ST2] = Pt * Pt + Qt * Qt;
  if (!hessian) return;
  const int* ws = d.line_wsrc + 8 * l;
  double wPf = ws[0] >= 0 ? lam[ws[0]] : 0.0;
  double wQf = ws[1] >= 0 ? lam[ws[1]] : 0.0;
  double wPt = ws[2] >= 0 ? lam[ws[2]] : 0.0;
  double wQt = ws[3] >= 0 ? lam[ws[3]] : 0.0;
  if (ws[4] >= 0) wQf += y[ws[4]];
  if (ws[5] >= 0) wQt += y[ws[5]];
  const int f = d.lf[l], t = d.lt[l];
  if (f == d.ref || t == d.ref) {
    // Pg_ref = P_ref + Pd_ref is a function of the state: its multiplier and
    // the derivative of its cost weight the Hessian of P_ref
    const double pg_ref = ref_injection(d, x, u) + d.src[d.src_u + d.nu + d.ref];
    const double w = y[0] + d.c2_ref * 2.0 * d.base * d.base * pg_ref + d.c1_ref * d.base;
    if (f == d.ref) wPf += w; else wPt += w;
  }
  const double ysf = ws[6] >= 0 ? y[ws[6]] : 0.0;
  const double yst = ws[7] >= 0 ? y[ws[7]] : 0.0;
  const double cPf = wPf + 2.0 * ysf * Pf, cQf = wQf + 2.0 * ysf * Qf;
  const double cPt = wPt + 2.0 * yst * Pt, cQt = wQt + 2.0 * yst * Qt;
  double* h = d.hl + (size_t)HL_STRIDE * l;
  int idx = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b, ++idx) {
      double v = cPf * HPf[idx] + cQf * HQf[idx] + cPt * HPt[idx] + cQt * HQt[idx];
      v += 2.0 * ysf * (gPf[a] * gPf[b] + gQf[a] * gQf[b]);
      v += 2.0 * yst * (gPt[a] * gPt[b] + gQt[a] * gQt[b]);
      h[idx] = v;
    }
}

__global__ void __launch_bounds__(kBlock) k_gather(int n, const int* __restrict__ ptr,
                                                  const int* __restrict__ idx,
                                                  const double* __restrict__ coef,
                                                  const double* __restrict__ cst,
                                                  const double* __restrict__ src,
                                                  double* __restrict__ dst) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double acc = cst[e];
  for (int t = ptr[e]; t < ptr[e + 1]; ++t) acc += coef[t] * src[idx[t]];
  dst[e] = acc;
}

// K = W + diag(Sigma_u, Sigma_x) + A^T diag(Sigma_s) A on the fixed pattern.
// The reference generator's quadratic cost adds 2 c2 base^2 grad P_ref
// grad P_ref^T, i.e. it enlarges the weight of A's first row.
__global__ void __launch_bounds__(kBlock) k_assemble_k(DevNet d, const double* sig_x,
                                                      const double* sig_u,
                                                      const double* sig_s) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d.nnz_k) return;
  double acc = 0.0;
  for (int t = d.kg_hl_ptr[e]; t < d.kg_hl_ptr[e + 1]; ++t) acc += d.hl[d.kg_hl_idx[t]];
  const double* av = d.dst + d.d_a;
  for (int t = d.kg_ata_ptr[e]; t < d.kg_ata_ptr[e + 1]; ++t) {
    const int j = d.kg_row[t];
    const double w = sig_s[j] + (j == 0 ? d.cost_rank1 : 0.0);
    acc += av[d.kg_a1[t]] * av[d.kg_a2[t]] * w;
  }
  const int v = d.kg_diag[e];
  if (v >= 0) {
    const int s = d.sig_map[v];
    acc += (s < d.nu ? sig_u[s] : sig_x[s - d.nu]) + d.k_cdiag[v];
  }
  d.kval[e] = acc;
}

__global__ void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------- refactorisation
// One work-group; each wave factors one row at a time (rows of a level are
// independent). The row is staged in LDS; for each lower entry (i, k) in
// increasing k: l = a_ik / u_kk, then a_ij -= l * u_kj over row k of U, the
// lanes of the wave taking distinct j. Rows of U read here were finished in
// earlier levels.
constexpr int kRefWaves = 16;

__global__ void __launch_bounds__(64 * kRefWaves) k_refactor(DevNet d) {
  extern __shared__ double rowbuf_all[];
  double* lu = d.dst + d.d_lu;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  double* rowbuf = rowbuf_all + (size_t)wave * d.max_row;
  for (int lev = 0; lev < d.rf_nlev; ++lev) {
    const int s0 = d.rf_lev_ptr[lev], s1 = d.rf_lev_ptr[lev + 1];
    for (int slot = s0 + wave; slot < s1; slot += kRefWaves) {
      const int i = d.rf_rows[slot];
      const int rp0 = d.lu_ptr[i], rp1 = d.lu_ptr[i + 1], rd = d.lu_diag[i];
      double amax = 0.0;
      for (int t = lane; t < rp1 - rp0; t += 64) {
        const double v = lu[rp0 + t];
        rowbuf[t] = v;
        amax = fmax(amax, fabs(v));
      }
      for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
      __builtin_amdgcn_wave_barrier();
      for (int p = rp0; p < rd; ++p) {
        const double l = rowbuf[p - rp0] / lu[d.lu_diag[d.lu_col[p]]];
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) rowbuf[p - rp0] = l;
        for (int o = d.rf_kptr[p] + lane; o < d.rf_kptr[p + 1]; o += 64)
          rowbuf[d.rf_dst[o] - rp0] -= l * lu[d.rf_src[o]];
        __builtin_amdgcn_wave_barrier();
      }
      for (int t = lane; t < rp1 - rp0; t += 64) lu[rp0 + t] = rowbuf[t];
      if (lane == 0) {
        const double piv = rowbuf[rd - rp0];
        if (!(fabs(piv) > 1e-14 * amax)) {
          d.status[2] = 1;
          d.status[3] = i;
        }
      }
    }
    __syncthreads();
  }
}

// Copy the refactorised values into the four sweep layouts (level-ordered
// entries, reciprocal pivots).
__global__ void __launch_bounds__(kBlock) k_transcribe(DevNet d) {
  const double* lu = d.dst + d.d_lu;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  const DevSweep* sw[4] = {&d.sl, &d.su, &d.sut, &d.slt};
  for (int s = 0; s < 4; ++s) {
    const DevSweep& w = *sw[s];
    for (int t = tid; t < w.nnz; t += stride) w.val[t] = lu[w.src[t]];
    if (w.dinv)
      for (int t = tid; t < d.nx; t += stride) w.dinv[t] = 1.0 / lu[w.diag_src[t]];
  }
}

// rt = [r1 ; r2] + A^T (Sigma_s r5 - r3), in w = [u ; x internal] order.
__global__ void __launch_bounds__(kBlock) k_rtilde(DevNet d, const double* r, const double* sig_s) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= d.nw) return;
  const double* r1 = r;
  const double* r2 = r + d.nu;
  const double* r3 = r2 + d.nx;
  const double* r5 = r3 + d.m + d.nx;
  const double* av = d.dst + d.d_a;
  double acc = v < d.nu ? r1[v] : r2[d.perm[v - d.nu]];
  for (int e = d.acsc_ptr[v]; e < d.acsc_ptr[v + 1]; ++e) {
    const int j = d.acsc_row[e];
    acc += av[d.acsc_from[e]] * (sig_s[j] * r5[j] - r3[j]);
  }
  d.rt[v] = acc;
}

// ------------------------------------------------- condensation pipeline
// One level-ordered triangular sweep over a panel X (rows x W, W contiguous).
// Rows of one level are independent; work items are (row, column) pairs with
// the column fastest so that neighbouring lanes share matrix entries.
template <int W>
__device__ __forceinline__ void sweep(const DevSweep& s, double* X) {
  const int tid = threadIdx.x, T = blockDim.x;
  for (int lev = 0; lev < s.nlev; ++lev) {
    const int s0 = s.lev_ptr[lev], s1 = s.lev_ptr[lev + 1];
    const int n = (s1 - s0) * W;
    for (int item = tid; item < n; item += T) {
      const int slot = s0 + item / W, c = item % W;
      const int row = s.rows[slot];
      double acc = X[row * W + c];
      for (int e = s.ptr[slot]; e < s.ptr[slot + 1]; ++e) acc -= s.val[e] * X[s.col[e] * W + c];
      if (s.dinv) acc *= s.dinv[slot];
      X[row * W + c] = acc;
    }
    __syncthreads();
  }
}

enum { MODE_COLUMNS = 0, MODE_RECOVER = 1 };

// Columns [col0 + blockIdx.x * W, ...) of the condensed matrix (Section 3.3):
//   Z   = -G_x^{-1} G_u V          (L then U sweep; V = identity columns)
//   H   =  K [V ; Z]               (one sparse product over all nu + nx rows)
//   Psi =  G_x^{-T} H_x            (U^T then L^T sweep)
//   out =  H_u - G_u^T Psi         (column of K_cond)
// Column nu (if requested) is the condensed right-hand side: V = 0, Z = -G_x^{-1} r4,
// H += rt, and rhs = -out. In MODE_RECOVER (one column): V = p_u,
// Z = -G_x^{-1}(r4 + G_u p_u) = p_x, H += rt, Psi = -p_lambda.
template <int W, bool LDS>
__global__ void __launch_bounds__(kBlock) k_condense(DevNet d, int col0, int col_end, int mode,
                                                    const double* r, const double* vin,
                                                    double* K, long ldk, double* rhs,
                                                    double* p_out) {
  extern __shared__ double panel_lds[];
  const int nw = d.nw, nu = d.nu, nx = d.nx;
  double* P = LDS ? panel_lds : d.panel + (size_t)blockIdx.x * 2 * nw * W;
  double* H = P + (size_t)nw * W;
  const int jc0 = col0 + blockIdx.x * W;
  const int tid = threadIdx.x, T = blockDim.x;
  const double* gu = d.dst + d.d_gu;
  const double* r4 = r ? r + d.nu + d.nx + d.m : nullptr;
  for (int i = tid; i < nw * W; i += T) P[i] = 0.0;
  __syncthreads();
  for (int c = 0; c < W; ++c) {
    const int j = jc0 + c;
    if (j >= col_end) break;
    if (mode == MODE_RECOVER) {
      for (int v = tid; v < nu; v += T) P[v * W + c] = vin[v];
      for (int i = tid; i < nx; i += T) {
        double acc = r4[d.perm[i]];
        for (int e = d.gu_ptr[i]; e < d.gu_ptr[i + 1]; ++e) acc += gu[e] * vin[d.gu_col[e]];
        P[(nu + i) * W + c] = -acc;
      }
    } else if (j < nu) {
      if (tid == 0) P[j * W + c] = 1.0;
      for (int e = d.gucsc_ptr[j] + tid; e < d.gucsc_ptr[j + 1]; e += T)
        P[(nu + d.gucsc_row[e]) * W + c] = -gu[d.gucsc_from[e]];
    } else {
      for (int i = tid; i < nx; i += T) P[(nu + i) * W + c] = -r4[d.perm[i]];
    }
  }
  __syncthreads();
  sweep<W>(d.sl, P + nu * W);
  sweep<W>(d.su, P + nu * W);
  for (int item = tid; item < nw * W; item += T) {
    const int v = item / W, c = item % W;
    double acc = 0.0;
    for (int e = d.k_ptr[v]; e < d.k_ptr[v + 1]; ++e) acc += d.kval[e] * P[d.k_col[e] * W + c];
    const int j = jc0 + c;
    if (mode == MODE_RECOVER || j == nu) acc += d.rt[v];
    H[item] = acc;
  }
  __syncthreads();
  if (mode == MODE_RECOVER) {
    double* px = p_out + nu;
    for (int i = tid; i < nx; i += T) {
      const double z = P[(nu + i) * W];
      px[d.perm[i]] = z;
      d.pw[nu + i] = z;
    }
    for (int v = tid; v < nu; v += T) {
      d.pw[v] = vin[v];
      p_out[v] = vin[v];
    }
  }
  sweep<W>(d.sut, H + nu * W);
  sweep<W>(d.slt, H + nu * W);
  if (mode == MODE_RECOVER) {
    double* plam = p_out + nu + nx + d.m;
    for (int i = tid; i < nx; i += T) plam[d.perm[i]] = -H[(nu + i) * W];
    return;
  }
  for (int item = tid; item < nu * W; item += T) {
    const int q = item % nu, c = item / nu;
    const int j = jc0 + c;
    if (j >= col_end) continue;
    double acc = H[q * W + c];
    for (int e = d.gucsc_ptr[q]; e < d.gucsc_ptr[q + 1]; ++e)
      acc -= gu[d.gucsc_from[e]] * H[(nu + d.gucsc_row[e]) * W + c];
    if (j < nu)
      K[(size_t)j * ldk + q] = acc;
    else
      rhs[q] = -acc;
  }
}

// p_s = -r5 - A p,  p_y = -r3 - Sigma_s p_s   (p in w order from the recovery)
__global__ void __launch_bounds__(kBlock) k_finish_step(DevNet d, const double* r,
                                                       const double* sig_s, double* p) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= d.m) return;
  const double* r3 = r + d.nu + d.nx;
  const double* r5 = r3 + d.m + d.nx;
  const double* av = d.dst + d.d_a;
  double ap = 0.0;
  for (int e = d.a_ptr[j]; e < d.a_ptr[j + 1]; ++e) ap += av[e] * d.pw[d.a_col[e]];
  const double ps = -r5[j] - ap;
  p[d.nu + d.nx + j] = ps;
  p[d.nu + 2 * d.nx + d.m + j] = -r3[j] - sig_s[j] * ps;
}

__global__ void __launch_bounds__(kBlock) k_objective(DevNet d, const double* u,
                                                     const double* c2, const double* c1,
                                                     const double* c0, const int* pg_u,
                                                     double* f) {
  __shared__ double part[kBlock];
  double acc = 0.0;
  for (int g = threadIdx.x; g < d.ng; g += blockDim.x) {
    const double pg = g == d.ref_gen ? d.dst[d.d_h] : u[pg_u[g]];
    const double mw = d.base * pg;
    acc += c2[g] * mw * mw + c1[g] * mw + c0[g];
  }
  part[threadIdx.x] = acc;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if (threadIdx.x < s) part[threadIdx.x] += part[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) *f = part[0];
}

// --------------------------------------------------------- dense Cholesky
__global__ void k_symmetrize(double* K, long ld, int n) {
  const int i = blockIdx.x * 16 + threadIdx.x;
  const int j = blockIdx.y * 16 + threadIdx.y;
  if (i >= n || j >= i) return;
  const double v = 0.5 * (K[(size_t)j * ld + i] + K[(size_t)i * ld + j]);
  K[(size_t)j * ld + i] = v;
  K[(size_t)i * ld + j] = v;
}

constexpr int NB = 32;   // panel width of the blocked Cholesky

// Panel step k0 of a right-looking blocked Cholesky of the lower triangle of
// A + delta I, with the forward substitution L y = b folded in (b is a work
// copy whose rows below the panel receive b_i -= L_ik y_k). Block 0 owns the
// diagonal block and writes y_k; block t >= 1 owns rows [k0 + t NB, ...).
// Every block factors the (already updated) diagonal block and solves for
// y_k redundantly in LDS, so the panel needs no second launch.
__global__ void __launch_bounds__(1024) k_potrf_panel(double* A, long ld, int n, int k0,
                                                     double delta, double* b, double* y,
                                                     int* status) {
  if (status[0] != 0) return;
  __shared__ double L[NB][NB + 1];
  __shared__ double X[NB][NB + 1];
  __shared__ double yk[NB];
  const int tid = threadIdx.x;
  const int ti = tid % NB, tj = tid / NB;   // 32 x 32 threads
  const int bsz = min(NB, n - k0);
  {
    double v = 0.0;
    if (ti < bsz && tj < bsz && ti >= tj) v = A[(size_t)(k0 + tj) * ld + k0 + ti];
    if (ti == tj && ti < bsz) v += delta;
    L[ti][tj] = v;
  }
  __syncthreads();
  for (int j = 0; j < bsz; ++j) {
    const double djj = L[j][j];
    if (!(djj > 0.0)) {
      if (blockIdx.x == 0 && tid == 0) {
        status[0] = 1;
        status[1] = k0 + j;
      }
      return;   // uniform: every thread read the same pivot
    }
    const double s = sqrt(djj);
    __syncthreads();
    if (tj == 0 && ti > j && ti < bsz) L[ti][j] /= s;
    __syncthreads();
    if (tj > j && ti >= tj && ti < bsz) L[ti][tj] -= L[ti][j] * L[tj][j];
    if (tid == 0) L[j][j] = s;
    __syncthreads();
  }
  // y_k = L_kk^{-1} b_k (one wave, lane j owns row j)
  if (tid < 64) {
    const int lane = tid;
    const double bj = lane < bsz ? b[k0 + lane] : 0.0;
    double acc = 0.0, mine = 0.0;
    for (int c = 0; c < bsz; ++c) {
      const double val = lane < bsz ? (bj - acc) / L[lane][lane] : 0.0;
      const double yc = __shfl(val, c);
      if (lane == c) mine = yc;
      if (lane > c && lane < bsz) acc += L[lane][c] * yc;
    }
    if (lane < bsz) yk[lane] = mine;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    if (ti < bsz && tj < bsz && ti >= tj) A[(size_t)(k0 + tj) * ld + k0 + ti] = L[ti][tj];
    if (tid < bsz) y[k0 + tid] = yk[tid];
    return;
  }
  const int r0 = k0 + blockIdx.x * NB;
  const int rb = min(NB, n - r0);
  X[ti][tj] = (ti < rb && tj < bsz) ? A[(size_t)(k0 + tj) * ld + r0 + ti] : 0.0;
  __syncthreads();
  // X L^T = A_ik, column by column
  for (int j = 0; j < bsz; ++j) {
    if (tj == 0 && ti < rb) X[ti][j] /= L[j][j];
    __syncthreads();
    if (tj > j && tj < bsz && ti < rb) X[ti][tj] -= X[ti][j] * L[tj][j];
    __syncthreads();
  }
  if (ti < rb && tj < bsz) A[(size_t)(k0 + tj) * ld + r0 + ti] = X[ti][tj];
  if (tj == 0 && ti < rb) {
    double acc = 0.0;
    for (int c = 0; c < bsz; ++c) acc += X[ti][c] * yk[c];
    b[r0 + ti] -= acc;
  }
}

// Trailing update A[i, j] -= sum_c L[i, c] L[j, c] over the panel columns
// [k0, k0 + NB) for the lower tiles of the trailing matrix, 32 x 32 tiles.
__global__ void __launch_bounds__(256) k_syrk(double* A, long ld, int n, int k0, int* status) {
  if (status[0] != 0) return;
  const int k1 = k0 + NB;
  // triangular tile index -> (ti, tj), tj <= ti
  int t = blockIdx.x, ti = 0;
  while (t > ti) {
    t -= ti + 1;
    ++ti;
  }
  const int tj = t;
  const int i0 = k1 + ti * 32, j0 = k1 + tj * 32;
  __shared__ double Ai[32][NB + 1];
  __shared__ double Aj[32][NB + 1];
  const int tid = threadIdx.x;
  for (int e = tid; e < 32 * NB; e += 256) {
    const int r = e % 32, c = e / 32;
    Ai[r][c] = (i0 + r < n) ? A[(size_t)(k0 + c) * ld + i0 + r] : 0.0;
    Aj[r][c] = (j0 + r < n) ? A[(size_t)(k0 + c) * ld + j0 + r] : 0.0;
  }
  __syncthreads();
  const int r = tid % 32, cq = tid / 32;   // each thread: row r, columns cq*4 .. cq*4+3
  double acc[4] = {0, 0, 0, 0};
  for (int c = 0; c < NB; ++c) {
    const double a = Ai[r][c];
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[q] += a * Aj[cq * 4 + q][c];
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int gi = i0 + r, gj = j0 + cq * 4 + q;
    if (gi < n && gj < n && gj <= gi) A[(size_t)gj * ld + gi] -= acc[q];
  }
}

// Backward substitution L^T x = y in one work-group (x stored into y).
__global__ void __launch_bounds__(256) k_trsv_lt(const double* A, long ld, int n, double* y,
                                                 const int* status) {
  if (status[0] != 0) return;
  extern __shared__ double xs[];
  __shared__ double part[4][64];
  const int tid = threadIdx.x;
  for (int i = tid; i < n; i += 256) xs[i] = y[i];
  __syncthreads();
  const int nblk = (n + 63) / 64;
  for (int jb = nblk - 1; jb >= 0; --jb) {
    const int j0 = jb * 64, j1 = min(n, j0 + 64);
    // rhs_j -= sum_{i >= j1} L[i, j] x_i
    {
      const int j = j0 + tid % 64, q = tid / 64;
      double acc = 0.0;
      if (j < j1)
        for (int i = j1 + q; i < n; i += 4) acc += A[(size_t)j * ld + i] * xs[i];
      part[q][tid % 64] = acc;
    }
    __syncthreads();
    if (tid < 64) {
      const int lane = tid, j = j0 + lane;
      double rhs = 0.0;
      if (j < j1) rhs = xs[j] - (part[0][lane] + part[1][lane] + part[2][lane] + part[3][lane]);
      // solve the diagonal block backwards: lane j owns x_j
      double acc = 0.0, mine = 0.0;
      for (int c = j1 - 1; c >= j0; --c) {
        const double val = j < j1 ? (rhs - acc) / A[(size_t)j * ld + j] : 0.0;
        const double xc = __shfl(val, c - j0);
        if (j == c) mine = xc;
        if (j < c) acc += A[(size_t)j * ld + c] * xc;
      }
      if (j < j1) xs[j] = mine;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += 256) y[i] = xs[i];
}

template <int W, bool LDS>
hipError_t launch_condense_t(const DevNet& d, int col0, int ncols, int mode, const double* r,
                             const double* vin, double* K, long ldk, double* rhs, double* p,
                             hipStream_t st) {
  const int nblk = (ncols + W - 1) / W;
  const size_t lds = LDS ? (size_t)2 * d.nw * W * sizeof(double) : 0;
  hipLaunchKernelGGL((k_condense<W, LDS>), dim3(nblk), dim3(kBlock), lds, st, d, col0,
                     col0 + ncols, mode, r, vin, K, ldk, rhs, p);
  return hipGetLastError();
}

template <bool LDS>
hipError_t dispatch_width(const DevNet& d, int col0, int ncols, int width, int mode,
                          const double* r, const double* vin, double* K, long ldk, double* rhs,
                          double* p, hipStream_t st) {
  switch (width) {
    case 1: return launch_condense_t<1, LDS>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    case 2: return launch_condense_t<2, LDS>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    case 3: return launch_condense_t<3, LDS>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    case 4: return launch_condense_t<4, LDS>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    case 8: return launch_condense_t<8, LDS>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    default: return hipErrorInvalidValue;
  }
}

inline int cdiv(long a, long b) { return int((a + b - 1) / b); }

}  // namespace

void prepare_lds_kernels(size_t bytes) {
  const void* fns[] = {
      reinterpret_cast<const void*>(&k_condense<1, true>),
      reinterpret_cast<const void*>(&k_condense<2, true>),
      reinterpret_cast<const void*>(&k_condense<3, true>),
      reinterpret_cast<const void*>(&k_condense<4, true>),
      reinterpret_cast<const void*>(&k_condense<8, true>)};
  for (const void* f : fns)
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  (void)hipGetLastError();
}

int max_lds_bytes() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
    return 65536;
  return v;
}

hipError_t launch_eval(const DevNet& d, const double* x, const double* u, const double* lam,
                       const double* y, bool hessian, hipStream_t st) {
  const int n = d.nl > d.nu ? d.nl : d.nu;
  hipLaunchKernelGGL(k_eval_lines, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, d, x, u, lam, y,
                     hessian ? 1 : 0);
  hipLaunchKernelGGL(k_gather, dim3(cdiv(d.d_total, kBlock)), dim3(kBlock), 0, st, d.d_total,
                     d.eg_ptr, d.eg_idx, d.eg_coef, d.eg_cst, (const double*)d.src, d.dst);
  return hipGetLastError();
}

hipError_t launch_assemble_k(const DevNet& d, const double* sig_x, const double* sig_u,
                             const double* sig_s, hipStream_t st) {
  hipLaunchKernelGGL(k_assemble_k, dim3(cdiv(d.nnz_k, kBlock)), dim3(kBlock), 0, st, d, sig_x,
                     sig_u, sig_s);
  return hipGetLastError();
}

hipError_t launch_refactor(const DevNet& d, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, d.status + 2, 2, 0);
  hipLaunchKernelGGL(k_refactor, dim3(1), dim3(64 * kRefWaves),
                     (size_t)kRefWaves * d.max_row * sizeof(double), st, d);
  hipLaunchKernelGGL(k_transcribe, dim3(64), dim3(kBlock), 0, st, d);
  return hipGetLastError();
}

hipError_t launch_rtilde(const DevNet& d, const double* r, const double* sig_s, hipStream_t st) {
  hipLaunchKernelGGL(k_rtilde, dim3(cdiv(d.nw, kBlock)), dim3(kBlock), 0, st, d, r, sig_s);
  return hipGetLastError();
}

hipError_t launch_condense(const DevNet& d, int col0, int ncols, int width, bool lds,
                           const double* r, double* K, long ldk, double* rhs, hipStream_t st) {
  if (lds)
    return dispatch_width<true>(d, col0, ncols, width, MODE_COLUMNS, r, nullptr, K, ldk, rhs,
                                nullptr, st);
  return dispatch_width<false>(d, col0, ncols, width, MODE_COLUMNS, r, nullptr, K, ldk, rhs,
                               nullptr, st);
}

hipError_t launch_recover(const DevNet& d, const double* pu, const double* r, double* p,
                          hipStream_t st) {
  const bool lds = (size_t)2 * d.nw * sizeof(double) <= (size_t)max_lds_bytes();
  if (lds)
    return dispatch_width<true>(d, 0, 1, 1, MODE_RECOVER, r, pu, nullptr, 0, nullptr, p, st);
  return dispatch_width<false>(d, 0, 1, 1, MODE_RECOVER, r, pu, nullptr, 0, nullptr, p, st);
}

hipError_t launch_finish_step(const DevNet& d, const double* r, const double* sig_s, double* p,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_finish_step, dim3(cdiv(d.m, kBlock)), dim3(kBlock), 0, st, d, r, sig_s, p);
  return hipGetLastError();
}

hipError_t launch_symmetrize(double* K, long ldk, int n, hipStream_t st) {
  hipLaunchKernelGGL(k_symmetrize, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0, st, K, ldk, n);
  return hipGetLastError();
}

hipError_t launch_cholesky_solve(double* K, long ldk, int n, double delta, double* b,
                                 double* y, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, status, 2, 0);
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nblk = cdiv(n - k0, NB);
    hipLaunchKernelGGL(k_potrf_panel, dim3(nblk), dim3(1024), 0, st, K, ldk, n, k0, delta, b,
                       y, status);
    const int rest = n - (k0 + NB);
    if (rest > 0) {
      const int nt = cdiv(rest, 32);
      hipLaunchKernelGGL(k_syrk, dim3(nt * (nt + 1) / 2), dim3(256), 0, st, K, ldk, n, k0, status);
    }
  }
  hipLaunchKernelGGL(k_trsv_lt, dim3(1), dim3(256), (size_t)n * sizeof(double), st,
                     (const double*)K, ldk, n, y, (const int*)status);
  return hipGetLastError();
}

hipError_t launch_eval_objective(const DevNet& d, const double* u, double* f, hipStream_t st) {
  hipLaunchKernelGGL(k_objective, dim3(1), dim3(kBlock), 0, st, d, u, d.c2, d.c1, d.c0, d.pg_u, f);
  return hipGetLastError();
}

}  // namespace rh
