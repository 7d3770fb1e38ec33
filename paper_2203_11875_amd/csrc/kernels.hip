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
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= d.kell_n) return;
  const int e = d.kell_pos[t];
  if (e < 0) {
    d.kell_val[t] = 0.0;
    return;
  }
  double acc = 0.0;
  for (int q = d.kg_hl_ptr[e]; q < d.kg_hl_ptr[e + 1]; ++q) acc += d.hl[d.kg_hl_idx[q]];
  const double* av = d.dst + d.d_a;
  for (int q = d.kg_ata_ptr[e]; q < d.kg_ata_ptr[e + 1]; ++q) {
    const int j = d.kg_row[q];
    const double w = sig_s[j] + (j == 0 ? d.cost_rank1 : 0.0);
    acc += av[d.kg_a1[q]] * av[d.kg_a2[q]] * w;
  }
  const int v = d.kg_diag[e];
  if (v >= 0) {
    const int sm = d.sig_map[v];
    acc += (sm < d.nu ? sig_u[sm] : sig_x[sm - d.nu]) + d.k_cdiag[v];
  }
  d.kell_val[t] = acc;
}

__global__ void k_fill_int(int* p, int n, int v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ------------------------------------------------------- refactorisation
// One work-group of 1024 threads walks the levels of the L sweep (rows of a
// level are independent). In each level, groups of lanes (a per-level power
// of two chosen by the analysis so that as many rows as the LDS allows are in
// flight) each factor one row: the row, the U entries its elimination reads
// (rows finished in earlier levels) and its pivot reciprocals are staged in
// LDS with all loads of the row in flight together; then for each lower entry
// (i, k) in increasing k: l = a_ik / u_kk and a_ij -= l * u_kj over row k of
// U, the lanes of the group taking distinct j. The reciprocal of the new
// pivot is kept for the rows that follow.
constexpr int kRefThreads = 1024;

__global__ void __launch_bounds__(kRefThreads) k_refactor(DevNet d) {
  extern __shared__ double ref_lds[];
  double* lu = d.dst + d.d_lu;
  for (int lev = 0; lev < d.rf_nlev; ++lev) {
    const int s0 = d.rf_lev_ptr[lev], s1 = d.rf_lev_ptr[lev + 1];
    const int* mt = d.rf_lmeta + 6 * lev;
    const int lanes = mt[0], stride = mt[1];
    const int groups = kRefThreads / lanes;
    const int g = threadIdx.x / lanes, lane = threadIdx.x & (lanes - 1);
    double* rowbuf = ref_lds + (size_t)g * stride;
    double* srcbuf = rowbuf + mt[2];
    double* pivbuf = rowbuf + mt[3];
    int* dstbuf = reinterpret_cast<int*>(rowbuf + mt[4]);
    int* kbuf = dstbuf + mt[5];
    for (int slot = s0 + g; slot < s1; slot += groups) {
      const int4 i0 = *reinterpret_cast<const int4*>(d.rf_info + 8 * slot);
      const int2 i1 = *reinterpret_cast<const int2*>(d.rf_info + 8 * slot + 4);
      const int i = i0.x, rp0 = i0.y, rp1 = i0.z, rd = i0.w, o0 = i1.x, nops = i1.y;
      const int nlow = rd - rp0;
      double amax = 0.0;
      for (int t = lane; t < rp1 - rp0; t += lanes) {
        const double v = lu[rp0 + t];
        rowbuf[t] = v;
        amax = fmax(amax, fabs(v));
      }
      for (int t = lane; t < nops; t += lanes) {
        srcbuf[t] = lu[d.rf_src[o0 + t]];
        dstbuf[t] = d.rf_dst_local[o0 + t];
      }
      for (int t = lane; t < nlow; t += lanes) pivbuf[t] = d.rinv[d.lu_col[rp0 + t]];
      for (int t = lane; t <= nlow; t += lanes) kbuf[t] = d.rf_kptr[rp0 + t] - o0;
      for (int off = lanes / 2; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
      __builtin_amdgcn_wave_barrier();
      for (int q = 0; q < nlow; ++q) {
        const double l = rowbuf[q] * pivbuf[q];
        __builtin_amdgcn_wave_barrier();
        if (lane == 0) rowbuf[q] = l;
        for (int t = kbuf[q] + lane; t < kbuf[q + 1]; t += lanes)
          rowbuf[dstbuf[t]] = fma(-l, srcbuf[t], rowbuf[dstbuf[t]]);
        __builtin_amdgcn_wave_barrier();
      }
      for (int t = lane; t < rp1 - rp0; t += lanes) lu[rp0 + t] = rowbuf[t];
      if (lane == 0) {
        const double piv = rowbuf[rd - rp0];
        d.rinv[i] = 1.0 / piv;
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
    for (int t = tid; t < w.ell_n; t += stride) w.ell_val[t] = w.ell_src[t] >= 0 ? lu[w.ell_src[t]] : 0.0;
    if (!w.unit)
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
// Work-group barrier. When every value exchanged between threads lives in
// LDS, only LDS operations need to complete before the barrier: global loads
// issued ahead of time (the next level's matrix entries) stay in flight.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <bool LDS>
__device__ __forceinline__ void block_sync() {
  if (LDS)
    lds_barrier();
  else
    __syncthreads();
}

// Level metadata of one sweep, staged in LDS at kernel start:
// [slot0, rows, base, len, log2(lanes)] per level.
constexpr int kMeta = 5;

__device__ __forceinline__ void stage_meta(const DevSweep& s, int* meta) {
  for (int l = threadIdx.x; l < s.nlev; l += blockDim.x) {
    meta[kMeta * l + 0] = s.lev_ptr[l];
    meta[kMeta * l + 1] = s.lev_ptr[l + 1] - s.lev_ptr[l];
    meta[kMeta * l + 2] = s.lev_base[l];
    meta[kMeta * l + 3] = s.lev_len[l];
    meta[kMeta * l + 4] = __ffs(s.lev_lanes[l]) - 1;
  }
}

// Entries of one level that a thread loads ahead of time: up to PF entries
// of its first row, that row's index and its reciprocal pivot.
constexpr int PF = 4;
struct LevelFetch {
  int col[PF];
  double val[PF];
  int row;
  double dinv;
};

__device__ __forceinline__ void fetch_level(const DevSweep& s, const int* m, LevelFetch& f) {
  // branch-free (addresses clamped, values masked) so that the number of
  // loads in flight is the same on every path and waits stay exact
  const int R = m[1], ls = m[4];
  const int g = threadIdx.x >> ls, lane = threadIdx.x & ((1 << ls) - 1);
  const bool live = g < R;
  const int base = m[2], Lm = m[3];
#pragma unroll
  for (int j = 0; j < PF; ++j) {
    const int k = lane + (j << ls);
    const bool ok = live && k < Lm;
    const int idx = ok ? base + k * R + g : 0;
    const int c = s.ell_col[idx];
    const double v = s.ell_val[idx];
    f.col[j] = ok ? c : 0;
    f.val[j] = ok ? v : 0.0;
  }
  const int q = live ? m[0] + g : 0;
  f.row = s.rows[q];
  f.dinv = s.dinv[q];
}

// One level of a triangular sweep over a panel X (rows x W, the W columns of
// a row contiguous). Rows of a level are independent. Each row is taken by a
// group of 2^ls lanes (chosen per level from its longest row); each lane
// accumulates a strided share of the row's entries for all W columns, and the
// group reduces with cross-lane shuffles. The summation order depends only on
// the level structure, so results repeat bitwise and do not depend on W.
template <int W, bool LDS>
__device__ __forceinline__ void sweep_level(const DevSweep& s, const int* m, const LevelFetch& f,
                                            double* X) {
  const int s0 = m[0], R = m[1], base = m[2], Lm = m[3], ls = m[4];
  if (Lm == 0 && s.unit) return;    // nothing changes in this level: no barrier needed
  const int S = 1 << ls;
  const int g = threadIdx.x >> ls, lane = threadIdx.x & (S - 1), G = blockDim.x >> ls;
  for (int r = g; r < R; r += G) {
    double acc[W];
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] = 0.0;
    int row, k0;
    double dv;
    if (r == g) {
#pragma unroll
      for (int j = 0; j < PF; ++j) {
        const double* xc = X + f.col[j] * W;
#pragma unroll
        for (int c = 0; c < W; ++c) acc[c] = fma(f.val[j], xc[c], acc[c]);
      }
      row = f.row;
      dv = f.dinv;
      k0 = lane + PF * S;
    } else {
      row = s.rows[s0 + r];
      dv = s.dinv[s0 + r];
      k0 = lane;
    }
    for (int k = k0; k < Lm; k += S) {
      const int idx = base + k * R + r;
      const double v = s.ell_val[idx];
      const double* xc = X + s.ell_col[idx] * W;
#pragma unroll
      for (int c = 0; c < W; ++c) acc[c] = fma(v, xc[c], acc[c]);
    }
    for (int off = S >> 1; off > 0; off >>= 1)
#pragma unroll
      for (int c = 0; c < W; ++c) acc[c] += __shfl_xor(acc[c], off);
    if (lane == 0) {
#pragma unroll
      for (int c = 0; c < W; ++c) {
        X[row * W + c] = (X[row * W + c] - acc[c]) * dv;
      }
    }
  }
  block_sync<LDS>();
}

// A whole sweep, level by level. Entries come from the padded per-level
// layout, whose addresses need no row pointers, so the loads of level l+1
// are issued before level l is computed (two register sets used in turn, so
// the wait for one level's loads never waits for the next level's).
template <int W, bool LDS>
__device__ __forceinline__ void sweep(const DevSweep& s, const int* meta, double* X,
                                      long long* lt = nullptr) {
  LevelFetch a, b;
  const int n = s.nlev;
  fetch_level(s, meta, a);
  for (int lev = 0; lev < n; lev += 2) {
    if (lev + 1 < n) fetch_level(s, meta + kMeta * (lev + 1), b);
    sweep_level<W, LDS>(s, meta + kMeta * lev, a, X);
    if (lt && threadIdx.x == 0) lt[lev] = wall_clock64();
    if (lev + 1 >= n) break;
    if (lev + 2 < n) fetch_level(s, meta + kMeta * (lev + 2), a);
    sweep_level<W, LDS>(s, meta + kMeta * (lev + 1), b, X);
    if (lt && threadIdx.x == 0) lt[lev + 1] = wall_clock64();
  }
}

enum { MODE_COLUMNS = 0, MODE_RECOVER = 1 };

// Phase timestamp of work-group 0 (wall clock) when tracing is on.
__device__ __forceinline__ void tick(const DevNet& d, int k) {
  if (d.trace && blockIdx.x == 0 && threadIdx.x == 0) d.trace[k] = wall_clock64();
}

// Row kKRowBlock * bk + tid of H = K [V ; Z] (+ rt for the right-hand-side /
// recovery column), from the padded row-block layout of K.
template <int W>
__device__ __forceinline__ void hvp_row(const DevNet& d, const double* P, int bk, int tid,
                                        int jc0, int mode, double (&h)[W]) {
  const int v = bk * kKRowBlock + tid;
  const int base = d.kb_base[bk], len = d.kb_len[bk];
  double acc[W];
#pragma unroll
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
#pragma unroll 8
  for (int k = 0; k < len; ++k) {
    const int idx = base + k * kKRowBlock + tid;
    const double kv = d.kell_val[idx];
    const double* pc = P + d.kell_col[idx] * W;
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] = fma(kv, pc[c], acc[c]);
  }
  const double rt = (v < d.nw) ? d.rt[v] : 0.0;
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int j = jc0 + c;
    h[c] = (mode == MODE_RECOVER || j == d.nu) ? acc[c] + rt : acc[c];
  }
}

// Columns [col0 + blockIdx.x * W, ...) of the condensed matrix (Section 3.3):
//   Z   = -G_x^{-1} G_u V          (L then U sweep; V = identity columns)
//   H   =  K [V ; Z]               (one sparse product over all nu + nx rows)
//   Psi =  G_x^{-T} H_x            (U^T then L^T sweep)
//   out =  H_u - G_u^T Psi         (column of K_cond)
// Column nu (if requested) is the condensed right-hand side: V = 0, Z = -G_x^{-1} r4,
// H += rt, and rhs = -out. In MODE_RECOVER (one column): V = p_u,
// Z = -G_x^{-1}(r4 + G_u p_u) = p_x, H += rt, Psi = -p_lambda.
template <int W, bool LDS, int mode>
__global__ void __launch_bounds__(kBlock) k_condense(DevNet d, int col0, int col_end,
                                                    const double* r, const double* vin,
                                                    double* K, long ldk, double* rhs,
                                                    double* p_out) {
  extern __shared__ double panel_lds[];
  const int nw = d.nw, nu = d.nu, nx = d.nx;
  // LDS: one panel P (the Hessian product is held in registers and written
  // back over it); global: two panels P and H per work-group
  double* P = LDS ? panel_lds : d.panel + (size_t)blockIdx.x * 2 * nw * W;
  int* meta = reinterpret_cast<int*>(panel_lds + (LDS ? (size_t)nw * W : 0));
  int* m_sl = meta;
  int* m_su = m_sl + kMeta * d.sl.nlev;
  int* m_sut = m_su + kMeta * d.su.nlev;
  int* m_slt = m_sut + kMeta * d.sut.nlev;
  stage_meta(d.sl, m_sl);
  stage_meta(d.su, m_su);
  stage_meta(d.sut, m_sut);
  stage_meta(d.slt, m_slt);
  tick(d, 0);
  double* H = LDS ? P : P + (size_t)nw * W;
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
  tick(d, 1);
  sweep<W, LDS>(d.sl, m_sl, P + nu * W, (d.trace && blockIdx.x == 0) ? d.trace + 16 : nullptr);
  tick(d, 2);
  sweep<W, LDS>(d.su, m_su, P + nu * W);
  tick(d, 3);
  if (mode == MODE_COLUMNS) {
    // keep Z = S e_j (and d for the right-hand-side column) for the recovery
    for (int c = 0; c < W; ++c) {
      const int j = jc0 + c;
      if (j >= col_end) break;
      double* zc = d.zcols + (size_t)j * nx;
      for (int i = tid; i < nx; i += T) zc[i] = P[(nu + i) * W + c];
    }
  }
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
  // H = K [V ; Z]: thread t takes row kKRowBlock * b + t of every row block.
  // With the panel in LDS the rows are kept in registers until every thread
  // has read P, then written over it.
  if (LDS) {
    double hreg[kMaxRowBlocks][W];
#pragma unroll
    for (int bk = 0; bk < kMaxRowBlocks; ++bk) {
#pragma unroll
      for (int c = 0; c < W; ++c) hreg[bk][c] = 0.0;
      if (bk < d.kb_n) hvp_row<W>(d, P, bk, tid, jc0, mode, hreg[bk]);
    }
    block_sync<LDS>();
#pragma unroll
    for (int bk = 0; bk < kMaxRowBlocks; ++bk) {
      const int v = bk * kKRowBlock + tid;
      if (bk < d.kb_n && v < nw)
#pragma unroll
        for (int c = 0; c < W; ++c) H[v * W + c] = hreg[bk][c];
    }
    block_sync<LDS>();
  } else {
    for (int bk = 0; bk < d.kb_n; ++bk) {
      double h[W];
      hvp_row<W>(d, P, bk, tid, jc0, mode, h);
      const int v = bk * kKRowBlock + tid;
      if (v < nw)
#pragma unroll
        for (int c = 0; c < W; ++c) H[v * W + c] = h[c];
    }
    block_sync<LDS>();
  }
  tick(d, 4);
  sweep<W, LDS>(d.sut, m_sut, H + nu * W);
  tick(d, 5);
  sweep<W, LDS>(d.slt, m_slt, H + nu * W);
  tick(d, 6);
  if (mode == MODE_COLUMNS) {
    for (int c = 0; c < W; ++c) {
      const int j = jc0 + c;
      if (j >= col_end) break;
      double* pc = d.psicols + (size_t)j * nx;
      for (int i = tid; i < nx; i += T) pc[i] = H[(nu + i) * W + c];
    }
  }
  if (mode == MODE_RECOVER) {
    double* plam = p_out + nu + nx + d.m;
    for (int i = tid; i < nx; i += T) plam[d.perm[i]] = -H[(nu + i) * W];
    return;
  }
  for (int q = tid; q < nu; q += T) {
    double acc[W];
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] = H[q * W + c];
    for (int e = d.gucsc_ptr[q]; e < d.gucsc_ptr[q + 1]; ++e) {
      const double gv = gu[d.gucsc_from[e]];
      const double* hc = H + (nu + d.gucsc_row[e]) * W;
#pragma unroll
      for (int c = 0; c < W; ++c) acc[c] = fma(-gv, hc[c], acc[c]);
    }
#pragma unroll
    for (int c = 0; c < W; ++c) {
      const int j = jc0 + c;
      if (j >= col_end) break;
      if (j < nu)
        K[(size_t)j * ldk + q] = acc[c];
      else
        rhs[q] = -acc[c];
    }
  }
  tick(d, 7);
}

// Recovery from the stored columns: thread i (internal x index) of chunk ch
// sums the columns [ch * cw, (ch + 1) * cw) of Z and Psi against p_u; the
// partial sums are combined in a fixed order by k_recover_finish, so the
// result repeats bitwise.
constexpr int kRecChunks = 8;

__global__ void __launch_bounds__(kBlock) k_recover_partial(DevNet d, const double* pu) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ch = blockIdx.y;
  if (i >= d.nx) return;
  const int cw = (d.nu + kRecChunks - 1) / kRecChunks;
  const int j0 = ch * cw, j1 = min(d.nu, j0 + cw);
  double sz = 0.0, sp = 0.0;
#pragma unroll 4
  for (int j = j0; j < j1; ++j) {
    const double u = pu[j];
    sz = fma(d.zcols[(size_t)j * d.nx + i], u, sz);
    sp = fma(d.psicols[(size_t)j * d.nx + i], u, sp);
  }
  d.rpart[(size_t)ch * d.nx + i] = sz;
  d.rpart[(size_t)(kRecChunks + ch) * d.nx + i] = sp;
}

__global__ void __launch_bounds__(kBlock) k_recover_finish(DevNet d, double* p) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < d.nu) {
    d.pw[i] = p[i];
  }
  if (i >= d.nx) return;
  double sz = d.zcols[(size_t)d.nu * d.nx + i];
  double sp = d.psicols[(size_t)d.nu * d.nx + i];
  for (int ch = 0; ch < kRecChunks; ++ch) {
    sz += d.rpart[(size_t)ch * d.nx + i];
    sp += d.rpart[(size_t)(kRecChunks + ch) * d.nx + i];
  }
  d.pw[d.nu + i] = sz;
  p[d.nu + d.perm[i]] = sz;                         // p_x
  p[d.nu + d.nx + d.m + d.perm[i]] = -sp;           // p_lambda
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

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) |
                                                (unsigned long long)(unsigned)lo));
}

// Panel step k0 of a right-looking blocked Cholesky of the lower triangle of
// A + delta I, with the forward substitution L y = b folded in (b is a work
// copy whose rows below the panel receive b_i -= L_ik y_k). Block 0 owns the
// diagonal block and writes L_kk and y_k; block t >= 1 owns rows
// [k0 + t NB, ...) and writes L_ik = A_ik L_kk^{-T}. Every block factors the
// (already updated) diagonal block redundantly, so the panel needs one
// launch. 256 threads; thread (i, c0) keeps elements (i, c0 + 8 q), q < 4, of
// the diagonal block and of its row block in registers. A pivot costs two
// barriers: (A) the pivot value is published; every thread forms the
// reciprocal square root and the owners of column j scale it, divide the
// row block's column j and form y_j; (B) the scaled columns are published
// and every thread applies the rank-one updates.
constexpr int kPanelThreads = 256;
constexpr int kPanelQ = NB * NB / kPanelThreads;   // elements per thread (4)

__global__ void __launch_bounds__(kPanelThreads) k_potrf_panel(double* A, long ld, int n, int k0,
                                                              double delta, double* b, double* y,
                                                              int* status) {
  if (status[0] != 0) return;
  __shared__ double lcol[NB];   // column j of L_kk
  __shared__ double xcol[NB];   // column j of the row block's L_ik
  __shared__ double piv;
  __shared__ double yj;
  const int tid = threadIdx.x;
  const int ti = tid % NB, c0 = tid / NB;          // c0 in [0, 8)
  const int bsz = min(NB, n - k0);
  const int r0 = k0 + blockIdx.x * NB;
  const int rb = blockIdx.x ? min(NB, n - r0) : 0;
  double a[kPanelQ], x[kPanelQ];
#pragma unroll
  for (int q = 0; q < kPanelQ; ++q) {
    const int c = c0 + 8 * q;
    double v = 0.0;
    if (ti < bsz && c <= ti) v = A[(size_t)(k0 + c) * ld + k0 + ti];
    if (ti == c && ti < bsz) v += delta;
    a[q] = v;
    x[q] = (ti < rb && c < bsz) ? A[(size_t)(k0 + c) * ld + r0 + ti] : 0.0;
  }
  double bi = (c0 == 0 && ti < bsz) ? b[k0 + ti] : 0.0;
  double bacc = 0.0, yv = 0.0;
  if (tid == 0) piv = a[0];                         // element (0, 0)
  for (int j = 0; j < bsz; ++j) {
    __syncthreads();                                // (A)
    const double d = piv;
    if (!(d > 0.0)) {
      if (blockIdx.x == 0 && tid == 0) {
        status[0] = 1;
        status[1] = k0 + j;
      }
      return;   // uniform: every thread read the same pivot
    }
    const double rs = rsqrt(d);
#pragma unroll
    for (int q = 0; q < kPanelQ; ++q) {
      if (c0 + 8 * q == j) {
        if (ti >= j && ti < bsz) {
          a[q] = ti == j ? d * rs : a[q] * rs;      // column j of L
          lcol[ti] = a[q];
        }
        if (ti < rb) {
          x[q] *= rs;                               // x_ij / l_jj
          xcol[ti] = x[q];
        }
      }
    }
    if (c0 == 0 && ti == j) {
      yv = bi * rs;                                 // y_j = b_j / l_jj
      yj = yv;
    }
    __syncthreads();                                // (B)
    const double li = lcol[ti], xi = xcol[ti], yc = yj;
#pragma unroll
    for (int q = 0; q < kPanelQ; ++q) {
      const int c = c0 + 8 * q;
      if (c > j && c < bsz) {
        const double lc = lcol[c];
        if (c <= ti && ti < bsz) a[q] = fma(-li, lc, a[q]);
        if (ti < rb) x[q] = fma(-xi, lc, x[q]);
      }
      if (c == j + 1 && ti == j + 1) piv = a[q];    // next pivot, after its update
    }
    if (c0 == 0) {
      if (ti > j && ti < bsz) bi = fma(-li, yc, bi);
      if (ti < rb) bacc = fma(xi, yc, bacc);
    }
  }
  if (blockIdx.x == 0) {
#pragma unroll
    for (int q = 0; q < kPanelQ; ++q) {
      const int c = c0 + 8 * q;
      if (ti < bsz && c <= ti) A[(size_t)(k0 + c) * ld + k0 + ti] = a[q];
    }
    if (c0 == 0 && ti < bsz) y[k0 + ti] = yv;
    return;
  }
#pragma unroll
  for (int q = 0; q < kPanelQ; ++q) {
    const int c = c0 + 8 * q;
    if (ti < rb && c < bsz) A[(size_t)(k0 + c) * ld + r0 + ti] = x[q];
  }
  if (c0 == 0 && ti < rb) b[r0 + ti] -= bacc;
}

// Inverse of every NB x NB lower-triangular diagonal block of the factor
// (one work-group per block), for the blocked backward substitution:
// X = L_bb^{-1} column by column, right-looking over the rows of L_bb.
__global__ void __launch_bounds__(NB * NB) k_diag_inverse(const double* A, long ld, int n,
                                                         double* inv, const int* status) {
  if (status[0] != 0) return;
  __shared__ double L[NB][NB + 1];
  __shared__ double xr[NB];
  const int bk = blockIdx.x, k0 = bk * NB, bsz = min(NB, n - k0);
  const int ti = threadIdx.x % NB, tc = threadIdx.x / NB;   // element (row ti, column tc)
  L[ti][tc] = (ti < bsz && tc <= ti) ? A[(size_t)(k0 + tc) * ld + k0 + ti] : 0.0;
  double xv = (ti == tc && ti < bsz) ? 1.0 : 0.0;          // X = I, then forward elimination
  __syncthreads();
  for (int j = 0; j < bsz; ++j) {
    if (ti == j) {
      xv /= L[j][j];
      xr[tc] = xv;
    }
    __syncthreads();
    if (ti > j && ti < bsz) xv = fma(-L[ti][j], xr[tc], xv);
    __syncthreads();
  }
  inv[(size_t)bk * NB * NB + tc * NB + ti] = (ti < bsz && tc < bsz) ? xv : 0.0;   // column-major
}

typedef double d4_t __attribute__((ext_vector_type(4)));

// Trailing update A[i, j] -= sum_c L[i, c] L[j, c] over the panel columns
// [k0, k0 + NB) for the lower 32 x 32 tiles of the trailing matrix, on FP64
// MFMA (16x16x4). Four waves per tile, one 16 x 16 quadrant each. Operand
// layout of v_mfma_f64_16x16x4f64: A[i][k] in lane i + 16 k, B[k][j] in lane
// j + 16 k, D[i][j] in lane j + 16 (i % 4), register i / 4.
__global__ void __launch_bounds__(256) k_syrk(double* A, long ld, int n, int k0, int* status) {
  if (status[0] != 0) return;
  const int k1 = k0 + NB;
  int t = blockIdx.x, ti = 0;
  while (t > ti) {
    t -= ti + 1;
    ++ti;
  }
  const int tj = t;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int qi = wave / 2, qj = wave % 2;
  if (ti == tj && qi < qj) return;            // strictly upper quadrant of a diagonal tile
  const int ri = k1 + ti * 32 + qi * 16;      // first row of the quadrant
  const int cj = k1 + tj * 32 + qj * 16;      // first column of the quadrant
  const int li = lane % 16, kk = lane / 16;
  const bool rok = ri + li < n, cok = cj + li < n;
  d4_t acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int s4 = 0; s4 < NB / 4; ++s4) {
    const size_t col = (size_t)(k0 + 4 * s4 + kk) * ld;
    const double av = rok ? A[col + ri + li] : 0.0;
    const double bv = cok ? A[col + cj + li] : 0.0;
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
  }
  const int j = cj + li;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int i = ri + 4 * r + kk;
    if (i < n && j < n && j <= i) A[(size_t)j * ld + i] -= acc[r];
  }
}

// Backward substitution L^T x = y in one work-group (x written over y), by
// NB-row blocks from the bottom: rhs_b = y_b - sum_{i below} L_ib^T x_i (dot
// products over contiguous columns of L, coalesced, no sequential chain),
// then x_b = L_bb^{-T} rhs_b with the inverted diagonal block.
__global__ void __launch_bounds__(256) k_trsv_lt(const double* A, long ld, int n, double* y,
                                                 const double* inv, const int* status) {
  if (status[0] != 0) return;
  extern __shared__ double xs[];
  __shared__ double red[NB][65];
  __shared__ double rhsb[NB];
  const int tid = threadIdx.x, lane = tid % 64, wave = tid / 64;
  for (int i = tid; i < n; i += 256) xs[i] = y[i];
  __syncthreads();
  const int nblk = (n + NB - 1) / NB;
  for (int bk = nblk - 1; bk >= 0; --bk) {
    const int j0 = bk * NB, j1 = min(n, j0 + NB);
    // each wave takes NB/4 columns with independent accumulators
    {
      double acc[NB / 4];
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) acc[q] = 0.0;
      for (int i = j1 + lane; i < n; i += 64) {
        const double xi = xs[i];
#pragma unroll
        for (int q = 0; q < NB / 4; ++q) {
          const int j = j0 + wave * (NB / 4) + q;
          if (j < j1) acc[q] = fma(A[(size_t)j * ld + i], xi, acc[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < NB / 4; ++q) red[wave * (NB / 4) + q][lane] = acc[q];
    }
    __syncthreads();
    if (tid < NB) {
      double sacc = 0.0;
      for (int l = 0; l < 64; ++l) sacc += red[tid][l];
      rhsb[tid] = j0 + tid < j1 ? xs[j0 + tid] - sacc : 0.0;
    }
    __syncthreads();
    if (tid < NB && j0 + tid < j1) {
      // x_b = L_bb^{-T} rhs_b: row tid of L_bb^{-T} is column tid of L_bb^{-1}
      const double* iv = inv + (size_t)bk * NB * NB + (size_t)tid * NB;
      double v = 0.0;
      for (int c = 0; c < NB; ++c) v = fma(iv[c], rhsb[c], v);
      xs[j0 + tid] = v;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += 256) y[i] = xs[i];
}

}  // namespace
size_t condense_meta_bytes(const DevNet& d);
namespace {

template <int W, bool LDS>
hipError_t launch_condense_t(const DevNet& d, int col0, int ncols, int mode, const double* r,
                             const double* vin, double* K, long ldk, double* rhs, double* p,
                             hipStream_t st) {
  const int nblk = (ncols + W - 1) / W;
  const size_t lds = (LDS ? (size_t)d.nw * W * sizeof(double) : 0) + condense_meta_bytes(d);
  if (mode == MODE_RECOVER)
    hipLaunchKernelGGL((k_condense<W, LDS, MODE_RECOVER>), dim3(nblk), dim3(kBlock), lds, st, d,
                       col0, col0 + ncols, r, vin, K, ldk, rhs, p);
  else
    hipLaunchKernelGGL((k_condense<W, LDS, MODE_COLUMNS>), dim3(nblk), dim3(kBlock), lds, st, d,
                       col0, col0 + ncols, r, vin, K, ldk, rhs, p);
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

size_t condense_meta_bytes(const DevNet& d) {
  return sizeof(int) * kMeta * (size_t)(d.sl.nlev + d.su.nlev + d.sut.nlev + d.slt.nlev);
}

void prepare_lds_kernels(size_t bytes) {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_refactor),
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  const void* fns[] = {
      reinterpret_cast<const void*>(&k_condense<1, true, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<2, true, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<3, true, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<4, true, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<8, true, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, true, MODE_RECOVER>)};
  const void* gfns[] = {
      reinterpret_cast<const void*>(&k_condense<1, false, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<2, false, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<3, false, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<4, false, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<8, false, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, false, MODE_RECOVER>)};
  for (const void* f : fns)
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes));
  for (const void* f : gfns)
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
  hipLaunchKernelGGL(k_assemble_k, dim3(cdiv(d.kell_n, kBlock)), dim3(kBlock), 0, st, d, sig_x,
                     sig_u, sig_s);
  return hipGetLastError();
}

hipError_t launch_refactor(const DevNet& d, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, d.status + 2, 2, 0);
  hipLaunchKernelGGL(k_refactor, dim3(1), dim3(kRefThreads),
                     (size_t)d.rf_lds_doubles * sizeof(double), st, d);
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
  const bool lds = d.kb_n <= kMaxRowBlocks &&
      (size_t)d.nw * sizeof(double) + condense_meta_bytes(d) <= (size_t)max_lds_bytes();
  if (lds)
    return launch_condense_t<1, true>(d, 0, 1, MODE_RECOVER, r, pu, nullptr, 0, nullptr, p, st);
  return launch_condense_t<1, false>(d, 0, 1, MODE_RECOVER, r, pu, nullptr, 0, nullptr, p, st);
}

hipError_t launch_recover_stored(const DevNet& d, double* p, hipStream_t st) {
  hipLaunchKernelGGL(k_recover_partial, dim3(cdiv(d.nx, kBlock), kRecChunks), dim3(kBlock), 0, st,
                     d, (const double*)p);
  hipLaunchKernelGGL(k_recover_finish, dim3(cdiv(d.nx > d.nu ? d.nx : d.nu, kBlock)), dim3(kBlock),
                     0, st, d, p);
  return hipGetLastError();
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
                                 double* y, double* dinv, int* status, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, status, 2, 0);
  for (int k0 = 0; k0 < n; k0 += NB) {
    const int nblk = cdiv(n - k0, NB);
    hipLaunchKernelGGL(k_potrf_panel, dim3(nblk), dim3(kPanelThreads), 0, st, K, ldk, n, k0,
                       delta, b, y, status);
    const int rest = n - (k0 + NB);
    if (rest > 0) {
      const int nt = cdiv(rest, 32);
      hipLaunchKernelGGL(k_syrk, dim3(nt * (nt + 1) / 2), dim3(256), 0, st, K, ldk, n, k0, status);
    }
  }
  hipLaunchKernelGGL(k_diag_inverse, dim3(cdiv(n, NB)), dim3(NB * NB), 0, st, (const double*)K,
                     ldk, n, dinv, (const int*)status);
  hipLaunchKernelGGL(k_trsv_lt, dim3(1), dim3(256), (size_t)n * sizeof(double), st,
                     (const double*)K, ldk, n, y, (const double*)dinv, (const int*)status);
  return hipGetLastError();
}

hipError_t launch_eval_objective(const DevNet& d, const double* u, double* f, hipStream_t st) {
  hipLaunchKernelGGL(k_objective, dim3(1), dim3(kBlock), 0, st, d, u, d.c2, d.c1, d.c0, d.pg_u, f);
  return hipGetLastError();
}

}  // namespace rh
