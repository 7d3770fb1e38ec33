// HIP kernels (gfx950) of the condensation hot path:
//   derivative values on fixed patterns, static-pivot refactorisation of G_x,
//   the fused tangent-solve / Hessian-product / adjoint-solve pipeline that
//   builds K_cond column blocks, symmetrisation and the step recovery (the
//   dense Cholesky and its solves are in chol.hip).
#include <hip/hip_runtime.h>

#include <cmath>

#include "analysis.hpp"
#include "device.hpp"
#include "ipm.hpp"

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
__device__ __forceinline__ void k_eval_lines_body(const DevNet& d, const double* x, const double* u, const double* lam, const double* y, int hessian) {
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
  // slot k of line l at k nl + l: the lanes' stores are contiguous
  const size_t nl = d.nl;
  double* o = d.src + l;
  o[LF_PF * nl] = Pf;
  o[LF_QF * nl] = Qf;
  o[LF_PT * nl] = Pt;
  o[LF_QT * nl] = Qt;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    o[(LF_DPF + k) * nl] = gPf[k];
    o[(LF_DQF + k) * nl] = gQf[k];
    o[(LF_DPT + k) * nl] = gPt[k];
    o[(LF_DQT + k) * nl] = gQt[k];
    o[(LF_DSF2 + k) * nl] = 2.0 * (Pf * gPf[k] + Qf * gQf[k]);
    o[(LF_DST2 + k) * nl] = 2.0 * (Pt * gPt[k] + Qt * gQt[k]);
  }
  o[LF_SF2 * nl] = Pf * Pf + Qf * Qf;
  o[LF_ST2 * nl] = Pt * Pt + Qt * Qt;
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
  double* h = d.hl + l;   // entry idx at idx nl + l
  int idx = 0;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = a; b < 4; ++b, ++idx) {
      double v = cPf * HPf[idx] + cQf * HQf[idx] + cPt * HPt[idx] + cQt * HQt[idx];
      v += 2.0 * ysf * (gPf[a] * gPf[b] + gQf[a] * gQf[b]);
      v += 2.0 * yst * (gPt[a] * gPt[b] + gQt[a] * gQt[b]);
      h[idx * nl] = v;
    }
}
__global__ void __launch_bounds__(kBlock) k_eval_lines(DevNet d, const double* x, const double* u, const double* lam, const double* y, int hessian) {
  k_eval_lines_body(d, x, u, lam, y, hessian);
}

__device__ __forceinline__ void k_gather_body(int n, const int* __restrict__ ptr, const int* __restrict__ idx, const double* __restrict__ coef, const double* __restrict__ cst, const double* __restrict__ src, double* __restrict__ dst) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  double acc = cst[e];
  for (int t = ptr[e]; t < ptr[e + 1]; ++t) acc += coef[t] * src[idx[t]];
  dst[e] = acc;
}
__global__ void __launch_bounds__(kBlock) k_gather(int n, const int* __restrict__ ptr, const int* __restrict__ idx, const double* __restrict__ coef, const double* __restrict__ cst, const double* __restrict__ src, double* __restrict__ dst) {
  k_gather_body(n, ptr, idx, coef, cst, src, dst);
}

// K = W + diag(Sigma_u, Sigma_x) + A^T diag(Sigma_s) A on the fixed pattern.
// The reference generator's quadratic cost adds 2 c2 base^2 grad P_ref
// grad P_ref^T, i.e. it enlarges the weight of A's first row.
__device__ __forceinline__ void k_assemble_k_body(const DevNet& d, const double* sig_x, const double* sig_u, const double* sig_s) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d.nnz_k) return;
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
  d.kstr[d.kdst[e]] = acc;
}
// sig_s_keep (optional): receives a copy of sig_s (m entries) for the
// recovery after the solve.
__global__ void __launch_bounds__(kBlock) k_assemble_k(DevNet d, const double* sig_x, const double* sig_u, const double* sig_s,
                                                       double* sig_s_keep) {
  if (sig_s_keep)
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < d.m; i += gridDim.x * blockDim.x)
      sig_s_keep[i] = sig_s[i];
  k_assemble_k_body(d, sig_x, sig_u, sig_s);
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

// Level lev of the staged refactorisation: the work-group's row groups take
// the level's rows first_group + g, first_group + g + group_stride, ...
__device__ __forceinline__ void refactor_staged_level(const DevNet& d, int lev, int first_group,
                                                      int group_stride) {
  extern __shared__ double ref_lds[];
  double* lu = d.dst + d.d_lu;
  const int s0 = d.rf_lev_ptr[lev], s1 = d.rf_lev_ptr[lev + 1];
  const int* mt = d.rf_lmeta + 6 * lev;
  const int lanes = mt[0], stride = mt[1];
  const int g = threadIdx.x / lanes, lane = threadIdx.x & (lanes - 1);
  double* rowbuf = ref_lds + (size_t)g * stride;
  double* srcbuf = rowbuf + mt[2];
  double* pivbuf = rowbuf + mt[3];
  int* dstbuf = reinterpret_cast<int*>(rowbuf + mt[4]);
  int* kbuf = dstbuf + mt[5];
  for (int slot = s0 + first_group + g; slot < s1; slot += group_stride) {
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
}

__device__ __forceinline__ void k_refactor_body(const DevNet& d) {
  for (int lev = 0; lev < d.rf_nlev; ++lev) {
    const int groups = kRefThreads / d.rf_lmeta[6 * lev];
    refactor_staged_level(d, lev, 0, groups);
    __syncthreads();
  }
}
// One level of the staged refactorisation over ceil(rows / groups)
// work-groups (large networks: a level's rows need more row groups than one
// work-group's LDS holds); the level's rows only read rows of earlier
// levels, written by earlier launches.
__device__ __forceinline__ void k_refactor_level_staged_body(const DevNet& d, int lev) {
  const int groups = kRefThreads / d.rf_lmeta[6 * lev];
  refactor_staged_level(d, lev, blockIdx.x * groups, groups * gridDim.x);
}
__global__ void __launch_bounds__(kRefThreads) k_refactor_level_staged(DevNet d, int lev) {
  k_refactor_level_staged_body(d, lev);
}
__global__ void __launch_bounds__(kRefThreads) k_refactor(DevNet d) {
  k_refactor_body(d);
}

// Copy the refactorised values into the sweeps' lane blocks (entries,
// reciprocal pivots of the writing lanes) and the G_u values into the G_u^T
// record stream.
__device__ __forceinline__ void k_transcribe_body(const DevNet& d) {
  const double* lu = d.dst + d.d_lu;
  const double* gu = d.dst + d.d_gu;
  const int tid = blockIdx.x * blockDim.x + threadIdx.x;
  const int stride = gridDim.x * blockDim.x;
  for (int t = tid; t < d.tr_n; t += stride) d.lblk[d.tr_dst[t]] = lu[d.tr_src[t]];
  for (int t = tid; t < d.trd_n; t += stride) d.lblk[d.trd_dst[t]] = 1.0 / lu[d.trd_src[t]];
  for (int e = tid; e < d.nnz_gu; e += stride) d.gstr[d.gdst[e]] = gu[e];
}
__global__ void __launch_bounds__(kBlock) k_transcribe(DevNet d) {
  k_transcribe_body(d);
}

// rt = [r1 ; r2] + A^T (Sigma_s r5 - r3), in w = [u ; x internal] order.
__device__ __forceinline__ void k_rtilde_body(const DevNet& d, const double* r, const double* sig_s) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= d.nw) return;
  if (!r) {
    d.rt[v] = 0.0;
    d.kstr[d.krt_dst[v]] = 0.0;
    return;
  }
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
  d.kstr[d.krt_dst[v]] = acc;   // the rt term of K row v in the condensation's stream
}
__global__ void __launch_bounds__(kBlock) k_rtilde(DevNet d, const double* r, const double* sig_s) {
  k_rtilde_body(d, r, sig_s);
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

__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) |
                                                (unsigned long long)(unsigned)lo));
}

// p[i] when ok, else 0, with the load itself unconditional (p[0] stands in):
// a load inside a lane-divergent branch makes the compiler wait for it at
// the end of the branch, which serialises a run of such loads.
__device__ __forceinline__ double ld_or0(const double* p, size_t i, bool ok) {
  const double v = p[ok ? i : 0];
  return ok ? v : 0.0;
}

// ------------------------------------------- wave-resident refactorisation
// Same row-by-row Doolittle elimination as k_refactor, with U and the pivot
// reciprocals of the finished rows resident in LDS and each row held in
// registers, one lane per LU entry (a wave per long row, a 16-lane row of
// the wave per short row). Step q of a row broadcasts the multiplier of its
// q-th lower entry (readlane across the wave, or DPP row_newbcast within
// 16 lanes) and every lane applies a_p -= l_q u_(k_q, col p), reading u from
// LDS at the packed index prepared by the analysis. Levels of the L sweep are
// separated by barriers; inside a level each wave runs its own list of tasks
// and loads the next task's values and indices while running the current one.
struct RwRec {
  int v[kRwRec];
};

struct RwSet {
  double init;
  int ipos, rcol, udst, drow, pos, nsteps, wide;
  int pk[kRwPacked];
};

// Loads a task record (uniform). The values are only made scalar where they
// are used, a task later: waiting for them here would also wait for the
// loads of the next task issued just before.
__device__ __forceinline__ void rw_rec_load(const DevNet& d, int wave, int k, int cnt, RwRec& R) {
  const int gi = k < cnt ? d.rw_wbeg[wave] + k : d.rw_ntask;   // past the end: the dummy record
  const int* r = d.rw_rec + (size_t)gi * kRwRec;
#pragma unroll
  for (int f = 0; f < kRwRec; ++f) R.v[f] = r[f];
}

// Per-segment value of a record field (4 consecutive ints), chosen by selects
// of register values (readfirstlane keeps them from being folded back into
// one indexed load, which would put the record in scratch memory).
__device__ __forceinline__ int rw_seg(const RwRec& R, int f, int seg) {
  const int v0 = __builtin_amdgcn_readfirstlane(R.v[f]);
  const int v1 = __builtin_amdgcn_readfirstlane(R.v[f + 1]);
  const int v2 = __builtin_amdgcn_readfirstlane(R.v[f + 2]);
  const int v3 = __builtin_amdgcn_readfirstlane(R.v[f + 3]);
  return seg == 0 ? v0 : seg == 1 ? v1 : seg == 2 ? v2 : v3;
}

__device__ __forceinline__ void rw_set_load(const DevNet& d, const RwRec& R, RwSet& X, int lane) {
  X.nsteps = __builtin_amdgcn_readfirstlane(R.v[1]);
  X.wide = __builtin_amdgcn_readfirstlane(R.v[2]);
  int seg = X.wide ? 0 : lane >> 4;
  const int p = X.wide ? lane : lane & 15;
  asm volatile("" : "+v"(seg));                // keep the selects (no indexed table)
  const int rp0 = rw_seg(R, 4, seg), len = rw_seg(R, 8, seg), nl = rw_seg(R, 12, seg);
  const bool active = p < len, lower = p < nl;
  X.ipos = active ? rp0 + p : -1;
  X.init = ld_or0(d.dst + d.d_lu, X.ipos, active);
  X.rcol = d.lu_col[lower ? rp0 + p : 0];      // used only where lower
  X.pos = lower ? p : -1;
  X.udst = active && p > nl ? rw_seg(R, 16, seg) + (p - nl - 1) : -1;
  X.drow = active && p == nl ? rw_seg(R, 20, seg) : -1;
  // packed steps: rows past the task's own read the 64-int block at the end
#pragma unroll
  for (int k = 0; k < kRwPacked; ++k) {
    const int o = __builtin_amdgcn_readfirstlane(2 * k < X.nsteps ? R.v[0] + k * 64
                                                                   : d.rw_lane_pad);
    X.pk[k] = d.rw_lane[o + lane];
  }
}

__device__ __forceinline__ double rw_u(const double* ulds, int pk, int half, int zslot) {
  const int ui = (pk >> (16 * half)) & 0xffff;
  return ulds[min(ui, zslot)];
}

template <int Q>
__device__ __forceinline__ void rw_steps16(double& acc, double r, const RwSet& X, int nsteps,
                                           const double (&u)[16]) {
  if constexpr (Q < 16) {
    if (Q >= nsteps) return;
    const long long b = __builtin_bit_cast(long long, acc * r);
    const int lo = __builtin_amdgcn_update_dpp(0, int(b), 0x150 + Q, 0xF, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), 0x150 + Q, 0xF, 0xF, false);
    const double l = __builtin_bit_cast(
        double, (long long)(((unsigned long long)(unsigned)hi << 32) | (unsigned)lo));
    if (X.pos == Q) acc = l;
    acc = fma(-l, u[Q], acc);
    rw_steps16<Q + 1>(acc, r, X, nsteps, u);
  }
}

__device__ __forceinline__ void rw_run(const DevNet& d, const RwSet& X, double* ulds,
                                       double* rinv, int lane) {
  const int zslot = d.rw_nnz_u;
  const int nsteps = __builtin_amdgcn_readfirstlane(X.nsteps);
  const int wide = __builtin_amdgcn_readfirstlane(X.wide);
  double acc = X.init;
  const double r = X.pos >= 0 ? rinv[X.rcol] : 0.0;
  double amax = fabs(acc);
  if (wide) {
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (8 * c >= nsteps) break;
      double u[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) u[s] = rw_u(ulds, X.pk[4 * c + s / 2], s & 1, zslot);
#pragma unroll
      for (int s = 0; s < 8; ++s) asm volatile("" : "+v"(u[s]));   // read them all up front
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int q = 8 * c + s;
        if (q >= nsteps) break;
        const double l = readlane_d(acc * r, q);
        if (X.pos == q) acc = l;
        acc = fma(-l, u[s], acc);
      }
    }
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
  } else {
    double u[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) u[s] = rw_u(ulds, X.pk[s / 2], s & 1, zslot);
#pragma unroll
    for (int s = 0; s < 16; ++s) asm volatile("" : "+v"(u[s]));    // read them all up front
    rw_steps16<0>(acc, r, X, nsteps, u);
    for (int off = 8; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
  }
  if (X.ipos >= 0) d.dst[d.d_lu + X.ipos] = acc;
  if (X.udst >= 0) ulds[X.udst] = acc;
  if (X.drow >= 0) {
    rinv[X.drow] = 1.0 / acc;
    if (!(fabs(acc) > 1e-14 * amax)) {
      d.status[2] = 1;
      d.status[3] = X.drow;
    }
  }
}

// rw_run with U from the LU values in global memory (the rows of earlier
// levels, finished by earlier launches) and the pivot reciprocals in
// d.rinv: the same operations in the same order, so the results equal the
// wave-resident kernel's bit for bit.
__device__ __forceinline__ void rw_run_global(const DevNet& d, const RwSet& X, int lu0, int lane,
                                              bool first) {
  const double* lu = d.dst + d.d_lu;
  const int* pos = d.rw_lanelu + lu0 + lane;
  const int nsteps = __builtin_amdgcn_readfirstlane(X.nsteps);
  const int wide = __builtin_amdgcn_readfirstlane(X.wide);
  double acc = X.init;
  // the lower entries of a level-1 row are rows of level 0, whose pivots are
  // their values (the launch writes their reciprocals for later levels)
  const double r = X.pos < 0 ? 0.0 : first ? 1.0 / lu[d.lu_diag[X.rcol]] : d.rinv[X.rcol];
  double amax = fabs(acc);
  if (wide) {
    for (int c = 0; c < nsteps; c += 8) {
      double u[8];
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int p = c + s < nsteps ? pos[(c + s) * 64] : -1;
        u[s] = ld_or0(lu, p < 0 ? 0 : p, p >= 0);
      }
#pragma unroll
      for (int s = 0; s < 8; ++s) {
        const int q = c + s;
        if (q >= nsteps) break;
        const double l = readlane_d(acc * r, q);
        if (X.pos == q) acc = l;
        acc = fma(-l, u[s], acc);
      }
    }
    for (int off = 32; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
  } else {
    double u[16];
#pragma unroll
    for (int s = 0; s < 16; ++s) {
      const int p = s < nsteps ? pos[s * 64] : -1;
      u[s] = ld_or0(lu, p < 0 ? 0 : p, p >= 0);
    }
    rw_steps16<0>(acc, r, X, nsteps, u);
    for (int off = 8; off > 0; off >>= 1) amax = fmax(amax, __shfl_xor(amax, off));
  }
  if (X.ipos >= 0) d.dst[d.d_lu + X.ipos] = acc;
  if (X.drow >= 0) {
    d.rinv[X.drow] = 1.0 / acc;
    if (!(fabs(acc) > 1e-14 * amax)) {
      d.status[2] = 1;
      d.status[3] = X.drow;
    }
  }
}

// Level lev (1 <= lev <= rw_split) of the refactorisation: one task per
// single-wave work-group, task blockIdx.x of wave blockIdx.y's list. The
// launch of level 1 also writes the pivot reciprocals of the rows of level 0
// (no elimination), which later levels read.
__device__ __forceinline__ void k_refactor_level_body(const DevNet& d, int lev) {
  const int lane = threadIdx.x;
  if (lev == 1) {
    const double* lu = d.dst + d.d_lu;
    const int nb = gridDim.x * gridDim.y;
    for (int q = (blockIdx.y * gridDim.x + blockIdx.x) * 64 + lane; q < d.rf_lev_ptr[1];
         q += nb * 64) {
      const int i = d.rf_rows[q];
      d.rinv[i] = 1.0 / lu[d.lu_diag[i]];
    }
  }
  const int w = blockIdx.y;
  const int* lend = d.rw_levend + (size_t)w * d.rw_nlev;
  const int k = lend[lev - 1] + blockIdx.x;
  if (k >= lend[lev]) return;
  const int cnt = d.rw_wbeg[w + 1] - d.rw_wbeg[w];
  RwRec R;
  RwSet X;
  rw_rec_load(d, w, k, cnt, R);
  rw_set_load(d, R, X, lane);
  rw_run_global(d, X, __builtin_amdgcn_readfirstlane(R.v[3]), lane, lev == 1);
}
__global__ void __launch_bounds__(64) k_refactor_level(DevNet d, int lev) {
  k_refactor_level_body(d, lev);
}

// Work-group 0 factors. Work-groups 8 h (h >= 1), dispatched to the same XCD
// as work-group 0, read the task tables and the values into that XCD's L2
// ahead of it and exit; the others exit at once.
__device__ __forceinline__ void k_refactor_wave_body(const DevNet& d, int split) {
  if (blockIdx.x != 0) {
    if (blockIdx.x % 8 != 0) return;
    const int h = blockIdx.x / 8 - 1, nh = gridDim.x / 8 - 1;
    const int nrec = (d.rw_ntask + 1) * kRwRec, nlane = d.rw_lane_pad + 64;
    int iacc = 0;
    double acc = 0.0;
    // 16-int (64-byte) pieces, interleaved over the helpers, in table order
    for (int t = (h * kRwWaves * 64 + threadIdx.x) * 16; t < nrec; t += nh * kRwWaves * 64 * 16)
      iacc += d.rw_rec[t];
    for (int t = (h * kRwWaves * 64 + threadIdx.x) * 16; t < nlane; t += nh * kRwWaves * 64 * 16)
      iacc += d.rw_lane[t];
    for (int t = (h * kRwWaves * 64 + threadIdx.x) * 8; t < d.nnz_lu; t += nh * kRwWaves * 64 * 8)
      acc += d.dst[d.d_lu + t];
    asm volatile("" :: "v"(acc), "v"(iacc));   // keeps the loads
    return;
  }
  extern __shared__ double rw_lds[];
  double* ulds = rw_lds;                       // U entries, then the zero slot
  double* rinv = rw_lds + d.rw_nnz_u + 1;      // reciprocal pivots by row
  int* levend = reinterpret_cast<int*>(rinv + d.nx);   // per wave: end of each level
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // optional profile: wall clock at the start, after level 0 and after
  // every later level
  long long* tr = d.trace && threadIdx.x == 0 ? d.trace + 127 : nullptr;
  if (tr) tr[0] = wall_clock64();
  const int cnt = d.rw_wbeg[wave + 1] - d.rw_wbeg[wave];
  // levels 1 .. split were factored by k_refactor_level (their rows are
  // final in global memory and their reciprocals in d.rinv)
  const int k0 = d.rw_levend[wave * d.rw_nlev + split];
  RwRec r0, r1;
  RwSet A, B;
  rw_rec_load(d, wave, k0, cnt, r0);
  rw_rec_load(d, wave, k0 + 1, cnt, r1);
  rw_set_load(d, r0, A, lane);
  if (threadIdx.x == 0) ulds[d.rw_nnz_u] = 0.0;
  for (int t = threadIdx.x; t < kRwWaves * d.rw_nlev; t += kRwWaves * 64) levend[t] = d.rw_levend[t];
  // level 0 (rows without lower entries keep their values) and the levels
  // factored before: U rows and pivot reciprocals into LDS
  const double* lu = d.dst + d.d_lu;
  const int nlev0 = d.rf_lev_ptr[1];
  for (int q = threadIdx.x; q < d.rf_lev_ptr[split + 1]; q += kRwWaves * 64) {
    const int i = d.rf_rows[q], rp0 = d.lu_ptr[i], rd = d.lu_diag[i], r1e = d.lu_ptr[i + 1];
    const int u0 = d.rw_ustart[i];
    double amax = 0.0;
    for (int p = rp0; p < r1e; ++p) {
      const double v = lu[p];
      amax = fmax(amax, fabs(v));
      if (p > rd) ulds[u0 + (p - rd - 1)] = v;
    }
    const double piv = lu[rd];
    rinv[i] = q < nlev0 ? 1.0 / piv : d.rinv[i];
    if (q < nlev0 && !(fabs(piv) > 1e-14 * amax)) {
      d.status[2] = 1;
      d.status[3] = i;
    }
  }
  lds_barrier();
  const int* lend = levend + wave * d.rw_nlev;
  if (tr) tr[1] = wall_clock64();
  int k = k0;
  for (int lev = split + 1; lev < d.rw_nlev; ++lev) {
    const int end = lend[lev];
    while (k < end) {
      if (((k - k0) & 1) == 0) {
        rw_set_load(d, r1, B, lane);
        rw_rec_load(d, wave, k + 2, cnt, r0);
        rw_run(d, A, ulds, rinv, lane);
      } else {
        rw_set_load(d, r0, A, lane);
        rw_rec_load(d, wave, k + 2, cnt, r1);
        rw_run(d, B, ulds, rinv, lane);
      }
      ++k;
    }
    lds_barrier();
    if (tr && lev < 128) tr[1 + lev] = wall_clock64();
  }
}
__global__ void __launch_bounds__(kRwWaves * 64) k_refactor_wave(DevNet d, int split) {
  k_refactor_wave_body(d, split);
}

// A wave takes one sweep step or one row block at a time (one thread per
// lane). The single-wave kernels (the G_x solves, condensation with more than
// one column per work-group or with panels in global memory) run kCondThreads.
constexpr int kCondThreads = kSweepThreads;
static_assert(kCondThreads == 64 && kKRowBlock == kCondThreads, "one lane per row of a block");
// Waves per condensation work-group (NW): one column with its panel in LDS
// may take kCondWaves or kCondWavesWide waves that share the panel (a
// sweep's same-level steps are spread over them, the record streams split
// into ranges of row blocks); every other shape runs one wave.
__host__ __device__ constexpr bool cond_waves_ok(int W, int PM, int NW) {
  return NW == 1 ||
         ((NW == kCondWavesPair || NW == kCondWaves || NW == kCondWavesWide) && W == 1 && PM != 0);
}
// step lists grouped for NW waves exist for these counts
__host__ __device__ constexpr bool cond_waves_grouped(int NW) {
  return NW == kCondWaves || NW == kCondWavesWide;
}

// Ordering of panel accesses between the steps of one wave. A wave's LDS
// operations complete in issue order, so for LDS panels a compiler-only
// fence is enough: it keeps the compiler from moving accesses across and
// emits no instruction (a wavefront-scope fence waits for the wave's LDS
// operations, lgkmcnt(0), once per sweep step); panels in global memory take
// a workgroup-scope fence, which waits for the stores.
template <bool LDS>
__device__ __forceinline__ void panel_sync() {
  if (LDS)
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
  else
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
}

// Step metadata of one sweep, staged in LDS at kernel start:
// {step index, log2 lanes per row, 0, 0} per step, then the idle step (every
// lane on padding that writes nothing).
__device__ __forceinline__ void stage_meta(const DevSweep& s, int4* meta) {
  const int4* src = reinterpret_cast<const int4*>(s.meta);
  for (int i = threadIdx.x; i <= s.nstep; i += blockDim.x) meta[i] = src[i];
}

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef unsigned u32x4 __attribute__((ext_vector_type(4)));

// What a lane loads ahead of time for one step: its kSweepPF values and
// panel offsets, reciprocal pivot, row offset and writer flag (every loaded
// dword is used, so that no register of an in-flight load is reused early,
// which would make the compiler wait for the load), and the step's uniform
// shape.
constexpr int PF = kSweepPF;
static_assert(PF == 8 && kStepDoubles == 7 * 128, "a step = 7 chunks of 64 x 16 bytes");
struct StepFetch {
  f64x2 v[PF / 2];
  u32x4 o[2];
  f64x2 piv;
  int ls;
};

// Seven 16-byte loads, each contiguous over the wave (chunk k of the step at
// k * kChunk doubles, lane t at 2 t).
__device__ __forceinline__ void fetch_step(const double* lblk, const int4 m, StepFetch& f) {
  const f64x2* b = reinterpret_cast<const f64x2*>(lblk + (size_t)m.x * kStepDoubles) + (threadIdx.x & 63);
#pragma unroll
  for (int k = 0; k < PF / 2; ++k) f.v[k] = b[k * (kChunk / 2)];
#pragma unroll
  for (int k = 0; k < 2; ++k) f.o[k] = reinterpret_cast<const u32x4*>(b + (4 + k) * (kChunk / 2))[0];
  f.piv = b[6 * (kChunk / 2)];
  f.ls = m.y;
}

// v + (v of lane `lane - SH` in the same 16-lane row; 0 at the row start)
template <int SH>
__device__ __forceinline__ double add_shr(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), 0x110 + SH, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), 0x110 + SH, 0xF, 0xF, true);
  return v + __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) |
                                                    (unsigned long long)(unsigned)lo));
}
// v + (lane 15 of the previous 16-lane row) in rows 1 and 3 (CTRL 0x142,
// rows 0xA), or + lane 31 in rows 2 and 3 (CTRL 0x143, rows 0xC).
template <int CTRL, int ROWS>
__device__ __forceinline__ double add_bcast(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, int(b), CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, int(b >> 32), CTRL, ROWS, 0xF, false);
  return v + __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) |
                                                    (unsigned long long)(unsigned)lo));
}

// Panel access by byte offset. LDS panels start at LDS address 0 (the
// condensation kernel has no static LDS, so its dynamic LDS begins there;
// the kernel checks this at start), so the offset is the address itself and
// costs no instruction; global panels use pb as a scalar base.
typedef __attribute__((address_space(3))) double lds_double;
template <bool LDS>
__device__ __forceinline__ double panel_ld(const char* pb, unsigned off) {
  if (LDS) return *reinterpret_cast<const lds_double*>((size_t)off);
  return *reinterpret_cast<const double*>(pb + off);
}
template <bool LDS>
__device__ __forceinline__ void panel_st(char* pb, unsigned off, double v) {
  if (LDS)
    *reinterpret_cast<lds_double*>((size_t)off) = v;
  else
    *reinterpret_cast<double*>(pb + off) = v;
}

// One step of a triangular sweep over the panels (byte offsets from pb; W
// columns of a row contiguous). The rows of a step are independent. Each row
// is taken by S = 2^ls consecutive lanes; a lane accumulates its entries for
// all W columns and the group sums with DPP shifts and row broadcasts, which
// leaves the row total in the group's last lane, the one that writes. The
// summation order depends only on the schedule, so results repeat bitwise and
// do not depend on W.
template <int W, bool LDS, int NW>
__device__ __forceinline__ void sweep_step(const StepFetch& f, char* pb) {
  double acc[W];
#pragma unroll
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
#pragma unroll
  for (int j = 0; j < PF; ++j) {
    const double v = f.v[j / 2][j % 2];
    const unsigned o = f.o[j / 4][j % 4];
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] = fma(v, panel_ld<LDS>(pb, o + 8 * c), acc[c]);
  }
  // row offset and writer flag (through a scalar: a bit cast of a vector
  // element subscript reads element 0)
  const double piv1 = f.piv.y;
  const unsigned long long rw = __builtin_bit_cast(unsigned long long, piv1);
  const unsigned row = unsigned(rw);
  double xr[W];
#pragma unroll
  for (int c = 0; c < W; ++c) xr[c] = panel_ld<LDS>(pb, row + 8 * c);
  // stages nested: a step leaves the tree with one branch after its last
  // stage (each column's sums in the same order as stage by stage)
  if (f.ls > 0) {
#pragma unroll
    for (int c = 0; c < W; ++c) acc[c] = add_shr<1>(acc[c]);
    if (f.ls > 1) {
#pragma unroll
      for (int c = 0; c < W; ++c) acc[c] = add_shr<2>(acc[c]);
      if (f.ls > 2) {
#pragma unroll
        for (int c = 0; c < W; ++c) acc[c] = add_shr<4>(acc[c]);
        if (f.ls > 3) {
#pragma unroll
          for (int c = 0; c < W; ++c) acc[c] = add_shr<8>(acc[c]);
          if (f.ls > 4) {
#pragma unroll
            for (int c = 0; c < W; ++c) acc[c] = add_bcast<0x142, 0xA>(acc[c]);
            if (f.ls > 5) {
#pragma unroll
              for (int c = 0; c < W; ++c) acc[c] = add_bcast<0x143, 0xC>(acc[c]);
            }
          }
        }
      }
    }
  }
  // the row's old value read (lgkmcnt(0)) before the writer branch, on every
  // path: otherwise the compiler keeps that read pending on the path that
  // skips the branch, and the next step's record loads, which reuse its
  // registers, wait for every LDS operation, the store just issued included
  if (LDS) __builtin_amdgcn_s_waitcnt(0xC07F);
  if (rw >> 32) {
#pragma unroll
    for (int c = 0; c < W; ++c)
      panel_st<LDS>(pb, row + 8 * c, (xr[c] - acc[c]) * f.piv.x);
  }
  // several waves: the steps of a group are done before the next group's
  // reads (global loads of later steps stay in flight)
  if constexpr (NW > 1)
    lds_barrier();
  else
    panel_sync<LDS>();
}

// A whole sweep, step by step. A step's lane block needs only the step's
// metadata (staged in LDS, read through lane registers), so the block of
// step k is requested while step k - kDepth + 1 is computed (kDepth register
// sets used in turn). Every pass of the loop requests one step and computes one:
// before the first step and after the last the sets hold the sweep's idle
// step (metadata entry n: every lane on a padding block that writes nothing),
// so the computation is unconditional and the compiler has no branch to sink
// a load into; and every load pending at the loop's back edge was issued in
// the same order on every path, so its waits stay exact (a step waits for its
// own block, never for the later steps').
constexpr int kDepth = 4;

template <int W, bool LDS, int NW = 1>
__device__ __forceinline__ void sweep(int n, const double* lblk, const int4* meta, char* pb) {
  if (n == 0) return;
  StepFetch f[kDepth];
  const int4 idle = meta[n];
#pragma unroll
  for (int j = 0; j < kDepth; ++j) fetch_step(lblk, idle, f[j]);
  // metadata in chunks of 64 steps: lane l holds step c + l (the idle step
  // past the end), a step's entry is read into scalar registers with lane
  // reads, so no memory latency falls inside the step loop
  for (int c = 0; c < n + kDepth - 1; c += 64) {
    const int4 mv = meta[min(c + (int)(threadIdx.x & 63), n)];
    // wait for it here (lgkmcnt(0)), once per chunk, so that no wait for it is
    // left at the head of the step loop
    __builtin_amdgcn_s_waitcnt(0xC07F);
    const int kend = min(c + 64, n + kDepth - 1);
    for (int k0 = c; k0 < kend; k0 += kDepth) {
#pragma unroll
      for (int j = 0; j < kDepth; ++j) {
        const int l = max(min(k0 + j, n) - c, 0);
        const int4 m{__builtin_amdgcn_readlane(mv.x, l), __builtin_amdgcn_readlane(mv.y, l), 0, 0};
        fetch_step(lblk, m, f[j]);
        sweep_step<W, LDS, NW>(f[(j + 1) % kDepth], pb);
      }
    }
  }
}

enum { MODE_COLUMNS = 0, MODE_RECOVER = 1 };

// Phase timestamp of work-group 0 (wall clock) when tracing is on.
__device__ __forceinline__ void tick(const DevNet& d, int k) {
  if (d.trace && blockIdx.x == 0 && threadIdx.x == 0) d.trace[k] = wall_clock64();
}

// Row-blocked record stream, blocks [b_lo, b_hi) on one wave: lane t owns
// stream position kKRowBlock * b + t of every block b; its records, kStreamBatch per batch
// (values, then panel byte offsets from pb; each 16-byte chunk contiguous
// over the wave), follow one another, block b covering records
// [end[b-1], end[b]). Per record acc += value * panel[offset]; at the end of
// a block flush(b, acc) and restart. Batch k is requested while batch
// k - kStreamDepth + 1 is computed (no prologue, as in the sweeps). end
// (LDS) and nblk are uniform.
constexpr int kStreamDepth = 4;
static_assert(kStreamBatch == 8 && kBatchDoubles == 6 * 128, "batch = 4 + 2 chunks of 64 x 16 bytes");
template <int W, bool LDS, class Flush>
__device__ __forceinline__ void row_stream(const double* str, const int* end_lds, int b_lo,
                                           int b_hi, const char* pb, Flush&& flush) {
  if (b_lo >= b_hi) return;
  const int ln = threadIdx.x & 63;
  // block ends through lane registers (refilled every 64 blocks)
  int ev = 0, ebase = -64;
  auto end = [&](int b) {
    if (b - ebase >= 64) {
      ebase = b;
      ev = end_lds[min(b + ln, b_hi - 1)];
    }
    return __builtin_amdgcn_readlane(ev, b - ebase);
  };
  // records [rec_start, rec_end) of blocks [b_lo, b_hi); the batch holding
  // rec_start may begin with records of the block before b_lo (a range of
  // another wave), which are left out
  // (read directly: the cached end() serves non-decreasing blocks only)
  const int rec_start = b_lo > 0 ? end_lds[b_lo - 1] : 0;
  const int rec_end = end_lds[b_hi - 1];
  const int first = rec_start / kStreamBatch;
  const int nbat = (rec_end + kStreamBatch - 1) / kStreamBatch - first;
  const f64x2* lane = reinterpret_cast<const f64x2*>(str) + ln + (size_t)first * (kBatchDoubles / 2);
  double acc[W];
#pragma unroll
  for (int c = 0; c < W; ++c) acc[c] = 0.0;
  int b = b_lo, e = end(b_lo);
  while (b < b_hi && e == rec_start) {   // blocks without records
    flush(b, acc);
    ++b;
    e = b < b_hi ? end(b) : 0x7fffffff;
  }
  if (nbat <= 0) return;
  f64x2 bv[kStreamDepth][kStreamBatch / 2];
  u32x4 bo[kStreamDepth][2];
#pragma unroll
  for (int j = 0; j < kStreamDepth; ++j) {
#pragma unroll
    for (int k = 0; k < kStreamBatch / 2; ++k) bv[j][k] = f64x2{0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 2; ++k) bo[j][k] = u32x4{0u, 0u, 0u, 0u};
  }
  // every pass requests one batch and computes one (zero records before the
  // first batch, repeats of the last after it: no flush falls there)
  for (int i0 = 0; i0 < nbat + kStreamDepth - 1; i0 += kStreamDepth) {
#pragma unroll
    for (int j = 0; j < kStreamDepth; ++j) {
      const f64x2* q = lane + (size_t)min(i0 + j, nbat - 1) * (kBatchDoubles / 2);
#pragma unroll
      for (int k = 0; k < kStreamBatch / 2; ++k) bv[j][k] = q[k * (kChunk / 2)];
#pragma unroll
      for (int k = 0; k < 2; ++k)
        bo[j][k] = reinterpret_cast<const u32x4*>(q + (4 + k) * (kChunk / 2))[0];
      const int cb = i0 + j - (kStreamDepth - 1);
      const int jj = (j + 1) % kStreamDepth;
      // the batch's panel reads first: a flush writes only the other panel
      // region (H for K [V; Z], P for G_u^T Psi), so none of them depends on
      // a flush, and all are in flight together
      double x[kStreamBatch][W];
#pragma unroll
      for (int r = 0; r < kStreamBatch; ++r)
#pragma unroll
        for (int c = 0; c < W; ++c) x[r][c] = panel_ld<LDS>(pb, bo[jj][r / 4][r % 4] + 8 * c);
      const int p0 = (first + cb) * kStreamBatch;
      if (p0 >= rec_start && p0 + kStreamBatch < e) {
        // no block ends inside the batch and all its records are this
        // range's: the same sums without a test per record
#pragma unroll
        for (int r = 0; r < kStreamBatch; ++r)
#pragma unroll
          for (int c = 0; c < W; ++c) acc[c] = fma(bv[jj][r / 2][r % 2], x[r][c], acc[c]);
        continue;
      }
#pragma unroll
      for (int r = 0; r < kStreamBatch; ++r) {
        const int p = p0 + r;
        const double v = p >= rec_start ? bv[jj][r / 2][r % 2] : 0.0;
#pragma unroll
        for (int c = 0; c < W; ++c) acc[c] = fma(v, x[r][c], acc[c]);
        while (p + 1 == e) {
          flush(b, acc);
#pragma unroll
          for (int c = 0; c < W; ++c) acc[c] = 0.0;
          ++b;
          e = b < b_hi ? end(b) : 0x7fffffff;
        }
      }
    }
  }
}

// The row blocks [first, last) of a record stream that wave `wave` of NW
// takes: contiguous ranges holding about equal numbers of records (end_lds:
// the blocks' record ends, in LDS).
template <int NW>
__device__ __forceinline__ int2 stream_range(const int* end_lds, int nblk) {
  if (NW == 1 || nblk <= 0) return int2{0, nblk};
  const int wave = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const long total = end_lds[nblk - 1];
  auto first_block = [&](int w) {
    if (w == 0) return 0;
    if (w >= NW) return nblk;
    const long target = total * w / NW;
    int cnt = 0;
    for (int b0 = 0; b0 < nblk; b0 += 64) {
      const int bb = b0 + ln;
      cnt += __popcll(__ballot(bb < nblk && end_lds[bb] <= target));
    }
    return cnt;
  };
  return int2{first_block(wave), first_block(wave + 1)};
}

// body(i, idx[i]) for i < n over the wave's lanes, the index loads of eight
// rounds issued together (clamped, so that none sits in a branch) before
// their bodies, whose stores could otherwise hold back the next loads.
template <class F>
__device__ __forceinline__ void indexed_loop(const int* idx, int n, F&& body) {
  const int T = blockDim.x;
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * T) {
    int ix[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) ix[u] = idx[min(i0 + u * T, n - 1)];
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u * T < n) body(i0 + u * T, ix[u]);
  }
}

// store(i, idx[i], load(i, idx[i])) for i < n over the work-group's threads: the
// index loads and then the value loads of eight rounds issued together
// (both clamped to row n - 1, whose index is valid, so that no load sits in
// a branch) before the stores.
template <class L, class S>
__device__ __forceinline__ void gather_loop(const int* idx, int n, L&& load, S&& store) {
  const int T = blockDim.x;
  for (int i0 = threadIdx.x; i0 < n; i0 += 8 * T) {
    int ix[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) ix[u] = idx[min(i0 + u * T, n - 1)];
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = load(min(i0 + u * T, n - 1), ix[u]);
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u * T < n) store(i0 + u * T, ix[u], v[u]);
  }
}

// Columns [col0 + blk * W, ...) of the condensed matrix (Section 3.3), one
// work-group of NW waves per tile (blk = the work-group's tile):
//   Z   = -G_x^{-1} G_u V          (L then U sweep; V = identity columns)
//   H   =  K [V ; Z]               (one sparse product over all nu + nx rows)
//   Psi =  G_x^{-T} H_x            (U^T then L^T sweep)
//   out =  H_u - G_u^T Psi         (column of K_cond)
// Column nu (if requested) is the condensed right-hand side: V = 0, Z = -G_x^{-1} r4,
// H += rt, and rhs = -out. In MODE_RECOVER (one column): V = p_u,
// Z = -G_x^{-1}(r4 + G_u p_u) = p_x, H += rt, Psi = -p_lambda.
// Panel (LDS or global, W doubles per row): P = [V; Z; indicator] (nw + 1
// rows; the indicator row is 1 in the right-hand-side / recovery column and
// multiplies each K row's rt term), then H over its first nw rows (in
// K-stream order: w row v at hpos[v]).
// PM (panel mode): 0 panels in global memory, 1 panels and sweep metadata in
// LDS, 2 panels in LDS with the sweep metadata read where it is (global
// memory, the same for every work-group), for networks whose panel alone
// fills the LDS. NW waves (several only for W = 1 with LDS panels) split the
// record streams and, per sweep, run it together or leave it to one wave.
template <int W, int PM, int NW, int mode>
__device__ __forceinline__ void k_condense_body(const DevNet& d, int blk, int col0, int col_end,
                                                const double* r, const double* vin, double* K,
                                                long ldk, double* rhs, double* p_out) {
  constexpr bool LDS = PM != 0;
  extern __shared__ double panel_lds[];
  if (LDS && (size_t)(lds_double*)panel_lds != 0) {   // the records assume LDS address 0
    if (blk == 0 && threadIdx.x == 0) d.status[4] = 1;
    return;
  }
  tick(d, 10);
  const int nw = d.nw, nu = d.nu, nx = d.nx;
  double* P = LDS ? panel_lds : d.panel + (size_t)blk * (nw + 1) * W;
  double* H = P;   // H replaces P after the Hessian product
  char* pb = reinterpret_cast<char*>(P);
  // step metadata of the four sweeps (with their idle steps), staged in LDS
  // unless PM == 2, then the block ends of the two record streams in LDS.
  // With NW waves a sweep whose bit is set in d.sweep_grouped runs on all of
  // them, as NW lists of groups (wave w taking list w); the other sweeps run
  // on one wave from the plain list while the other waves wait.
  static_assert(cond_waves_ok(W, PM, NW), "several waves: one column, panel in LDS");
  const int tid = threadIdx.x, T = 64 * NW, ln = tid & 63, wave = tid >> 6;
  auto csync = [&]() {
    if constexpr (NW > 1)
      __syncthreads();
    else
      panel_sync<LDS>();
  };
  int4* mlds = reinterpret_cast<int4*>(panel_lds + (LDS ? (size_t)(nw + 1) * W : 0));
  // the L sweep of an identity-column tile runs only the steps that can
  // change its panel (the reach of G_u's columns in L)
  const bool reach = mode == MODE_COLUMNS && d.lsk_ptr && col0 == 0;
  const int4* m_sw[4];
  int n_sw[4];
  bool grp[4];
  int* kb_end;
  constexpr int gi = NW == kCondWavesWide ? 1 : 0;   // which grouped lists
  const int jc0 = col0 + blk * W;
  const double* gu = d.dst + d.d_gu;
  const double* r4 = r ? r + d.nu + d.nx + d.m : nullptr;
  // The prologue's global reads go out in rounds that overlap: the first
  // G_u entries of the identity columns (three dependent reads: column
  // pointers, rows and sources, values) beside the staging of the step lists
  // and stream block ends (one read each, all requested before any store).
  int ge0[W], ge1[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int j = jc0 + c;
    const bool idc = mode == MODE_COLUMNS && j < nu && j < col_end;
    ge0[c] = idc ? d.gucsc_ptr[j] : 0;
    ge1[c] = idc ? d.gucsc_ptr[j + 1] : 0;
  }
  const int4* lsrc[4];
  int lcnt[4];
  {
    const DevSweep* sws[4] = {&d.sl, &d.su, &d.sut, &d.slt};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const DevSweep& sw = *sws[k];
      grp[k] = cond_waves_grouped(NW) && ((d.sweep_grouped >> k) & 1);
      const int4* src;
      int n;
      if (k == 0 && reach) {
        const int* ptr = grp[k] ? d.lsk_gptr[gi] : d.lsk_ptr;
        const int a = ptr[blk], e = ptr[blk + 1];
        src = reinterpret_cast<const int4*>(grp[k] ? d.lsk_gmeta[gi] : d.lsk_meta) + a;
        n = grp[k] ? (e - a) / NW - 1 : e - a - 1;
      } else {
        src = reinterpret_cast<const int4*>(grp[k] ? sw.gmeta[gi] : sw.meta);
        n = grp[k] ? sw.ngrp[gi] : sw.nstep;
      }
      n_sw[k] = n;
      lsrc[k] = src;
      lcnt[k] = (grp[k] ? NW : 1) * (n + 1);
    }
  }
  // first round of the staging: every list's element tid
  int4 v4[4];
  if constexpr (PM != 2) {
#pragma unroll
    for (int k = 0; k < 4; ++k) v4[k] = tid < lcnt[k] ? lsrc[k][tid] : int4{0, 0, 0, 0};
  }
  const int vk = tid < d.kb_n ? d.kb_end[tid] : 0;
  const int vg = tid < d.gt_nb ? d.gt_end[tid] : 0;
  int grw[W], gfr[W];
#pragma unroll
  for (int c = 0; c < W; ++c) {
    const int e = ge0[c] + tid;
    grw[c] = e < ge1[c] ? d.gucsc_row[e] : 0;
    gfr[c] = e < ge1[c] ? d.gucsc_from[e] : 0;
  }
  {
    const DevSweep* sws[4] = {&d.sl, &d.su, &d.sut, &d.slt};
    int4* slot = mlds;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int mine = grp[k] ? wave * (n_sw[k] + 1) : 0;
      if constexpr (PM == 2) {
        m_sw[k] = lsrc[k] + mine;
      } else {
        // the slot holds the sweep's whole list (a tile's reach list is no longer)
        if (tid < lcnt[k]) slot[tid] = v4[k];
        for (int i = tid + T; i < lcnt[k]; i += T) slot[i] = lsrc[k][i];
        m_sw[k] = slot + mine;
        slot += grp[k] ? NW * (sws[k]->ngrp[gi] + 1) : sws[k]->nstep + 1;
      }
    }
    kb_end = reinterpret_cast<int*>(PM == 2 ? mlds : slot);
  }
  double gvl[W];
#pragma unroll
  for (int c = 0; c < W; ++c) gvl[c] = ge0[c] + tid < ge1[c] ? gu[gfr[c]] : 0.0;
  // sweep k, then every wave waits for it; a sweep on one wave runs on wave
  // blk mod NW, so that the sweeping waves of the work-groups that share a CU
  // are spread over its SIMDs
  auto run_sweep = [&](int k) {
    if (grp[k])
      sweep<W, LDS, NW>(n_sw[k], d.lblk, m_sw[k], pb);
    else if (NW == 1 || wave == blk % NW)
      sweep<W, LDS, 1>(n_sw[k], d.lblk, m_sw[k], pb);
    csync();
  };
  int* gt_end = kb_end + d.kb_n;
  if (tid < d.kb_n) kb_end[tid] = vk;
  if (tid < d.gt_nb) gt_end[tid] = vg;
  for (int i = tid + T; i < d.kb_n; i += T) kb_end[i] = d.kb_end[i];
  for (int i = tid + T; i < d.gt_nb; i += T) gt_end[i] = d.gt_end[i];
  csync();
  tick(d, 0);
  for (int i = tid; i < (nw + 1) * W; i += T) P[i] = 0.0;
  csync();
  for (int c = 0; c < W; ++c) {
    const int j = jc0 + c;
    if (j >= col_end) break;
    if (mode == MODE_RECOVER || j == nu)
      if (tid == 0) P[nw * W + c] = 1.0;
    if (mode == MODE_RECOVER) {
      for (int v = tid; v < nu; v += T) P[v * W + c] = vin[v];
      // eight rows' dependent reads in flight at a time
      indexed_loop(d.perm, nx, [&](int i, int pi) {
        double acc = r4[pi];
        for (int e = d.gu_ptr[i]; e < d.gu_ptr[i + 1]; ++e) acc += gu[e] * vin[d.gu_col[e]];
        P[(nu + i) * W + c] = -acc;
      });
    } else if (j < nu) {
      if (tid == 0) P[j * W + c] = 1.0;
      if (ge0[c] + tid < ge1[c]) P[(nu + grw[c]) * W + c] = -gvl[c];
      for (int e = ge0[c] + tid + T; e < ge1[c]; e += T)
        P[(nu + d.gucsc_row[e]) * W + c] = -gu[d.gucsc_from[e]];
    } else {
      // the right-hand-side column, -r4 in the internal order (this tile's
      // fill is on the launch's critical path: eight rows' reads in flight)
      gather_loop(
          d.perm, nx, [&](int, int pi) { return r4[pi]; },
          [&](int i, int, double v) { P[(nu + i) * W + c] = -v; });
    }
  }
  csync();
  tick(d, 1);
  run_sweep(0);
  tick(d, 2);
  run_sweep(1);
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
  tick(d, 8);
  // H = K [V ; Z] (+ rt through the indicator row), row block by row block,
  // H rows in stream order; P is read to the end of the product, so H goes to
  // the tile's global scratch and then over P (its rows 0 .. nw - 1)
  double* scr = d.hscr + (size_t)blk * nw * W;
  const int2 kr = stream_range<NW>(kb_end, d.kb_n);
  row_stream<W, LDS>(d.kstr, kb_end, kr.x, kr.y, pb,
                     [&](int b, const double(&acc)[W]) {
                       const int p = b * kKRowBlock + ln;
                       if (p < nw)
#pragma unroll
                         for (int c = 0; c < W; ++c) scr[p * W + c] = acc[c];
                     });
  tick(d, 9);
  // the scratch stores complete (every wave's) before any wave reads them
  if constexpr (NW > 1)
    __syncthreads();
  else
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
  for (int i0 = tid; i0 < nw * W; i0 += 8 * T) {
    double v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = scr[min(i0 + k * T, nw * W - 1)];
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (i0 + k * T < nw * W) H[i0 + k * T] = v[k];
  }
  csync();
  tick(d, 4);
  run_sweep(2);
  tick(d, 5);
  run_sweep(3);
  tick(d, 6);
  if (mode == MODE_COLUMNS) {
    for (int c = 0; c < W; ++c) {
      const int j = jc0 + c;
      if (j >= col_end) break;
      double* pc = d.psicols + (size_t)j * nx;
      indexed_loop(d.hpos + nu, nx, [&](int i, int hp) { pc[i] = H[hp * W + c]; });
    }
  }
  if (mode == MODE_RECOVER) {
    double* plam = p_out + nu + nx + d.m;
    indexed_loop(d.hpos + nu, nx, [&](int i, int hp) { plam[d.perm[i]] = -H[hp * W]; });
    return;
  }
  // out = H_u - G_u^T Psi: the stream sums G_u^T Psi - H_u per control, written
  // to the K_cond column (rhs = -out for the right-hand-side column)
  const int2 gr = stream_range<NW>(gt_end, d.gt_nb);
  row_stream<W, LDS>(d.gstr, gt_end, gr.x, gr.y, pb,
                     [&](int b, const double(&acc)[W]) {
                       const int p = b * kKRowBlock + ln;
                       if (p < nu) {
                         const int q = d.grow[p];
#pragma unroll
                         for (int c = 0; c < W; ++c) {
                           const int j = jc0 + c;
                           if (j < nu)
                             K[(size_t)j * ldk + q] = -acc[c];
                           else if (j < col_end)
                             rhs[q] = acc[c];
                         }
                       }
                     });
  tick(d, 7);
}
template <int W, int PM, int NW, int mode>
__global__ void __launch_bounds__(64 * NW) k_condense(DevNet d, int col0, int col_end,
                                                          const double* r, const double* vin,
                                                          double* K, long ldk, double* rhs,
                                                          double* p_out) {
  // the last tile (the right-hand-side column's, whose full L sweep and dense
  // fill make it the longest) goes to the first work-group dispatched, on a
  // CU that no third work-group shares
  const int blk = blockIdx.x == 0 ? gridDim.x - 1 : blockIdx.x - 1;
  k_condense_body<W, PM, NW, mode>(d, blk, col0, col_end, r, vin, K, ldk, rhs, p_out);
}

// x = G_x^{-1} b (TRANS = 0: L then U sweep) or x = G_x^{-T} b (TRANS = 1:
// U^T then L^T sweep) with the factors of the last refactorisation, in one
// wave, on column 0 of a condensation panel (the records of the handle's
// panel width W); b and x in natural order. x = scale * solution, plus the
// old x if accumulate (a Newton step x -= G_x^{-1} g is scale -1).
template <int W, int PM, int TRANS>
__global__ void __launch_bounds__(kCondThreads) k_gx_solve(DevNet d, const double* b, double* x,
                                                          double scale, int accumulate) {
  constexpr bool LDS = PM != 0;
  extern __shared__ double panel_lds[];
  if (LDS && (size_t)(lds_double*)panel_lds != 0) {   // the records assume LDS address 0
    if (threadIdx.x == 0) d.status[4] = 1;
    return;
  }
  const int nw = d.nw, nu = d.nu, nx = d.nx, tid = threadIdx.x, T = kCondThreads;
  double* P = LDS ? panel_lds : d.panel;
  char* pb = reinterpret_cast<char*>(P);
  const DevSweep& s1 = TRANS ? d.sut : d.sl;
  const DevSweep& s2 = TRANS ? d.slt : d.su;
  const int4 *m1, *m2;
  if constexpr (PM == 2) {
    m1 = reinterpret_cast<const int4*>(s1.meta);
    m2 = reinterpret_cast<const int4*>(s2.meta);
  } else {
    int4* l1 = reinterpret_cast<int4*>(panel_lds + (LDS ? (size_t)(nw + 1) * W : 0));
    int4* l2 = l1 + s1.nstep + 1;
    stage_meta(s1, l1);
    stage_meta(s2, l2);
    m1 = l1;
    m2 = l2;
  }
  for (int i = tid; i < (nw + 1) * W; i += T) P[i] = 0.0;
  panel_sync<LDS>();
  if (TRANS)
    indexed_loop(d.hpos + nu, nx, [&](int i, int hp) { P[hp * W] = b[d.perm[i]]; });
  else
    gather_loop(
        d.perm, nx, [&](int, int pi) { return b[pi]; },
        [&](int i, int, double v) { P[(nu + i) * W] = v; });
  panel_sync<LDS>();
  sweep<W, LDS>(s1.nstep, d.lblk, m1, pb);
  sweep<W, LDS>(s2.nstep, d.lblk, m2, pb);
  panel_sync<LDS>();
  if (TRANS)
    indexed_loop(d.hpos + nu, nx, [&](int i, int hp) {
      const int k = d.perm[i];
      x[k] = (accumulate ? x[k] : 0.0) + scale * P[hp * W];
    });
  else
    gather_loop(
        d.perm, nx,
        [&](int i, int k) { return (accumulate ? x[k] : 0.0) + scale * P[(nu + i) * W]; },
        [&](int, int k, double v) { x[k] = v; });
}

// Recovery from the stored columns: thread i (internal x index) of chunk ch
// sums the columns [ch * cw, (ch + 1) * cw) of Z and Psi against p_u; the
// partial sums are combined in a fixed order by k_recover_finish, so the
// result repeats bitwise.
constexpr int kRecChunks = 8;

__device__ __forceinline__ void k_recover_partial_body(const DevNet& d, const double* pu) {
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
__global__ void __launch_bounds__(kBlock) k_recover_partial(DevNet d, const double* pu) {
  k_recover_partial_body(d, pu);
}

__device__ __forceinline__ void k_recover_finish_body(const DevNet& d, double* p) {
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
__global__ void __launch_bounds__(kBlock) k_recover_finish(DevNet d, double* p) {
  k_recover_finish_body(d, p);
}

// p_s = -r5 - A p,  p_y = -r3 - Sigma_s p_s   (p in w order from the recovery)
__device__ __forceinline__ void k_finish_step_body(const DevNet& d, const double* r, const double* sig_s, double* p) {
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
// hstat (optional, pinned host memory): receives the five status words,
// final once the solve's earlier kernels have run (this is its last).
__global__ void __launch_bounds__(kBlock) k_finish_step(DevNet d, const double* r, const double* sig_s, double* p,
                                                        int* hstat) {
  if (hstat && blockIdx.x == 0 && threadIdx.x < 5) hstat[threadIdx.x] = d.status[threadIdx.x];
  k_finish_step_body(d, r, sig_s, p);
}

__device__ __forceinline__ void k_objective_body(const DevNet& d, const double* u,
                                                 const double* c2, const double* c1,
                                                 const double* c0, const int* pg_u, double* f) {
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
__global__ void __launch_bounds__(kBlock) k_objective(DevNet d, const double* u,
                                                     const double* c2, const double* c1,
                                                     const double* c0, const int* pg_u,
                                                     double* f) {
  k_objective_body(d, u, c2, c1, c0, pg_u, f);
}
// objective of each active instance of a lockstep batch at its iterate
// (trial = 0: w into f[0]) or trial point (trial = 1: wt into f[1])
__global__ void __launch_bounds__(kBlock) k_objective_b(const DevNet* __restrict__ nets,
                                                       const IpmDev* __restrict__ ipms,
                                                       const double* sc, int trial) {
  if (sc[kIpmSc * blockIdx.z + IS_ACTIVE] == 0.0) return;
  const DevNet& d = cst(nets, blockIdx.z);
  const IpmDev& v = cst(ipms, blockIdx.z);
  k_objective_body(d, trial ? v.wt : v.w, d.c2, d.c1, d.c0, d.pg_u, v.f + trial);
}

// --------------------------------------------------------- dense Cholesky
// copy (optional, same layout): receives the symmetrised matrix, diagonal
// included (the saved copy for inertia-correction retries).
__device__ __forceinline__ void k_symmetrize_body(double* K, long ld, int n, double* copy = nullptr) {
  const int i = blockIdx.x * 16 + threadIdx.x;
  const int j = blockIdx.y * 16 + threadIdx.y;
  if (i >= n || j > i) return;
  if (j == i) {
    if (copy) copy[(size_t)i * ld + i] = K[(size_t)i * ld + i];
    return;
  }
  const double v = 0.5 * (K[(size_t)j * ld + i] + K[(size_t)i * ld + j]);
  K[(size_t)j * ld + i] = v;
  K[(size_t)i * ld + j] = v;
  if (copy) {
    copy[(size_t)j * ld + i] = v;
    copy[(size_t)i * ld + j] = v;
  }
}
__global__ void k_symmetrize(double* K, long ld, int n, double* copy) {
  k_symmetrize_body(K, ld, n, copy);
}

template <int W, int PM, int NW = 1>
hipError_t launch_condense_t(const DevNet& d, int col0, int ncols, int mode, const double* r,
                             const double* vin, double* K, long ldk, double* rhs, double* p,
                             hipStream_t st) {
  const int nblk = (ncols + W - 1) / W;
  const size_t lds = condense_lds_bytes(d, W, PM != 0, NW);
  if (mode == MODE_RECOVER)
    hipLaunchKernelGGL((k_condense<W, PM, NW, MODE_RECOVER>), dim3(nblk), dim3(64 * NW), lds, st,
                       d, col0, col0 + ncols, r, vin, K, ldk, rhs, p);
  else
    hipLaunchKernelGGL((k_condense<W, PM, NW, MODE_COLUMNS>), dim3(nblk), dim3(64 * NW), lds, st,
                       d, col0, col0 + ncols, r, vin, K, ldk, rhs, p);
  return hipGetLastError();
}

template <bool LDS>
hipError_t dispatch_width(const DevNet& d, int col0, int ncols, int width, int mode,
                          const double* r, const double* vin, double* K, long ldk, double* rhs,
                          double* p, hipStream_t st) {
  const int nwv = LDS ? d.cond_nw : 1;
  if (nwv != 1 && nwv != kCondWavesPair && nwv != kCondWaves && nwv != kCondWavesWide)
    return hipErrorInvalidValue;
  if (LDS && d.meta_global) {   // panel mode 2: one column per work-group only
    if (width != 1) return hipErrorInvalidValue;
    if (nwv == kCondWavesPair)
      return launch_condense_t<1, 2, kCondWavesPair>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    if (nwv == kCondWavesWide)
      return launch_condense_t<1, 2, kCondWavesWide>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    if (nwv == kCondWaves)
      return launch_condense_t<1, 2, kCondWaves>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    return launch_condense_t<1, 2>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
  }
  if (nwv > 1 && width != 1) return hipErrorInvalidValue;
  switch (width) {
    case 1:
      if constexpr (LDS) {
        if (nwv == kCondWavesPair)
          return launch_condense_t<1, 1, kCondWavesPair>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
        if (nwv == kCondWavesWide)
          return launch_condense_t<1, 1, kCondWavesWide>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
        if (nwv == kCondWaves)
          return launch_condense_t<1, 1, kCondWaves>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
      }
      return launch_condense_t<1, LDS>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    case 2: return launch_condense_t<2, LDS>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    case 3: return launch_condense_t<3, LDS>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    case 4: return launch_condense_t<4, LDS>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    case 8: return launch_condense_t<8, LDS>(d, col0, ncols, mode, r, vin, K, ldk, rhs, p, st);
    default: return hipErrorInvalidValue;
  }
}

inline int cdiv(long a, long b) { return int((a + b - 1) / b); }


// ------------------------------------------------------------ batches
// Batched launches: one launch serves every instance of a batch (instance =
// blockIdx.z unless noted); each instance's work uses its own DevNet and the
// same kernel bodies as the single-instance launches, so results are the
// same bit for bit.

__global__ void __launch_bounds__(kBlock) k_eval_lines_b(const DevNet* __restrict__ nets,
                                                        const BatchArg* __restrict__ a,
                                                        int hessian) {
  const int b = blockIdx.z;
  k_eval_lines_body(cst(nets, b), cst(a, b).x, cst(a, b).u, cst(a, b).lam, cst(a, b).y, hessian);
}
__global__ void __launch_bounds__(kBlock) k_gather_b(const DevNet* __restrict__ nets) {
  const DevNet& d = cst(nets, blockIdx.z);
  k_gather_body(d.d_total, d.eg_ptr, d.eg_idx, d.eg_coef, d.eg_cst, d.src, d.dst);
}
// per-instance vector copies kept by the handles (Sigma_s for the recovery,
// the right-hand side for the Cholesky solve): dst[i] = src[i], i < n
__global__ void __launch_bounds__(kBlock) k_copy_b(const BatchArg* __restrict__ a, int which) {
  const BatchArg& q = cst(a, blockIdx.z);
  const double* src = which == 0 ? q.sig_s : q.rhs;
  double* dst = which == 0 ? q.sig_s_keep : q.bwork;
  const int n = which == 0 ? q.m : q.nu;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    dst[i] = src[i];
}
__global__ void __launch_bounds__(kBlock) k_assemble_k_b(const DevNet* __restrict__ nets,
                                                        const BatchArg* __restrict__ a) {
  const int b = blockIdx.z;
  k_assemble_k_body(cst(nets, b), cst(a, b).sig_x, cst(a, b).sig_u, cst(a, b).sig_s);
}
__global__ void __launch_bounds__(kBlock) k_rtilde_b(const DevNet* __restrict__ nets,
                                                    const BatchArg* __restrict__ a) {
  const int b = blockIdx.z;
  k_rtilde_body(cst(nets, b), cst(a, b).r, cst(a, b).sig_s_keep);
}
// status[first .. first + count) = 0 for every instance
__global__ void k_clear_status_b(const DevNet* __restrict__ nets, int first, int count) {
  if ((int)threadIdx.x < count) cst(nets, blockIdx.z).status[first + threadIdx.x] = 0;
}
// Levels 1 .. rw_split of every instance with the wave-resident
// refactorisation, one launch per level for the batch (instances with fewer
// split levels skip), then the wave-resident kernel from each instance's split.
__global__ void __launch_bounds__(64) k_refactor_level_b(const DevNet* __restrict__ nets, int lev) {
  const DevNet& d = cst(nets, blockIdx.z);
  if (!d.rw_ok || lev > d.rw_split) return;
  k_refactor_level_body(d, lev);
}
__global__ void __launch_bounds__(kRwWaves * 64) k_refactor_wave_b(const DevNet* __restrict__ nets) {
  const DevNet& d = cst(nets, blockIdx.z);
  if (d.rw_ok) k_refactor_wave_body(d, d.rw_split);
}
__global__ void __launch_bounds__(kRefThreads) k_refactor_b(const DevNet* __restrict__ nets) {
  const DevNet& d = cst(nets, blockIdx.z);
  if (!d.rw_ok && !d.rf_per_level) k_refactor_body(d);
}
__global__ void __launch_bounds__(kRefThreads) k_refactor_level_staged_b(const DevNet* __restrict__ nets,
                                                                       int lev) {
  const DevNet& d = cst(nets, blockIdx.z);
  if (d.rw_ok || !d.rf_per_level || lev >= d.rf_nlev) return;
  k_refactor_level_staged_body(d, lev);
}
__global__ void __launch_bounds__(kBlock) k_transcribe_b(const DevNet* __restrict__ nets) {
  k_transcribe_body(cst(nets, blockIdx.z));
}
// work-group g takes tile tiles[g] = {instance, tile of W columns}
template <int W, int PM, int NW = 1>
__global__ void __launch_bounds__(64 * NW) k_condense_b(const DevNet* __restrict__ nets,
                                                            const BatchArg* __restrict__ a,
                                                            const int2* __restrict__ tiles) {
  const int2 t = tiles[blockIdx.x];
  const DevNet& d = cst(nets, t.x);
  const BatchArg& q = cst(a, t.x);
  k_condense_body<W, PM, NW, MODE_COLUMNS>(d, t.y, 0, d.nu + 1, q.r, nullptr, q.K, q.ldk, q.rhs,
                                       nullptr);
}
__global__ void k_symmetrize_b(const BatchArg* __restrict__ a) {
  const BatchArg& q = cst(a, blockIdx.z);
  k_symmetrize_body(q.K, q.ldk, q.nu);
}
__global__ void __launch_bounds__(kBlock) k_recover_partial_b(const DevNet* __restrict__ nets,
                                                             const BatchArg* __restrict__ a) {
  const int b = blockIdx.z;
  k_recover_partial_body(cst(nets, b), cst(a, b).p);
}
__global__ void __launch_bounds__(kBlock) k_recover_finish_b(const DevNet* __restrict__ nets,
                                                            const BatchArg* __restrict__ a) {
  const int b = blockIdx.z;
  k_recover_finish_body(cst(nets, b), cst(a, b).p);
}
// out[5 b + i] = status[i] of instance b, i < 5
__global__ void k_gather_status_b(const DevNet* __restrict__ nets, int* out) {
  if (threadIdx.x < 5) out[5 * blockIdx.z + threadIdx.x] = cst(nets, blockIdx.z).status[threadIdx.x];
}
__global__ void __launch_bounds__(kBlock) k_finish_step_b(const DevNet* __restrict__ nets,
                                                         const BatchArg* __restrict__ a) {
  const int b = blockIdx.z;
  k_finish_step_body(cst(nets, b), cst(a, b).r, cst(a, b).sig_s_keep, cst(a, b).p);
}

}  // namespace

size_t condense_lds_bytes(const DevNet& d, int width, bool lds_panels, int nwv) {
  static_assert(kSweepMeta == 4, "one int4 of metadata per step");
  // step lists: per sweep nstep + 1 entries, or nwv lists of ngrp + 1 for a
  // sweep that runs on all nwv waves (none when they are read from global
  // memory)
  size_t sweeps = 0;
  if (!(lds_panels && d.meta_global)) {
    const DevSweep* sws[4] = {&d.sl, &d.su, &d.sut, &d.slt};
    for (int k = 0; k < 4; ++k)
      sweeps += kSweepMeta * (cond_waves_grouped(nwv) && ((d.sweep_grouped >> k) & 1)
                                  ? (size_t)nwv * (sws[k]->ngrp[wave_index(nwv)] + 1)
                                  : (size_t)sws[k]->nstep + 1);
  }
  const size_t meta = sizeof(int) * (sweeps + (size_t)d.kb_n + (size_t)d.gt_nb);
  return (lds_panels ? (size_t)(d.nw + 1) * width * sizeof(double) : 0) + meta;
}

void prepare_lds_kernels() {
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_refactor),
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&k_refactor_wave),
                            hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  const void* fns[] = {
      reinterpret_cast<const void*>(&k_condense<1, 1, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<2, 1, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<3, 1, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<4, 1, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<8, 1, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, 1, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<2, 1, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<3, 1, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<4, 1, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<8, 1, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_gx_solve<1, 1, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<2, 1, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<3, 1, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<4, 1, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<8, 1, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<1, 1, 1>),
      reinterpret_cast<const void*>(&k_gx_solve<2, 1, 1>),
      reinterpret_cast<const void*>(&k_gx_solve<3, 1, 1>),
      reinterpret_cast<const void*>(&k_gx_solve<4, 1, 1>),
      reinterpret_cast<const void*>(&k_gx_solve<8, 1, 1>),
      reinterpret_cast<const void*>(&k_condense<1, 2, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, 2, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<1, 1, kCondWaves, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, 1, kCondWaves, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<1, 2, kCondWaves, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, 2, kCondWaves, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<1, 1, kCondWavesWide, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, 1, kCondWavesWide, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<1, 2, kCondWavesWide, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, 2, kCondWavesWide, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<1, 1, kCondWavesPair, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, 1, kCondWavesPair, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<1, 2, kCondWavesPair, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, 2, kCondWavesPair, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_gx_solve<1, 2, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<1, 2, 1>)};
  const void* gfns[] = {
      reinterpret_cast<const void*>(&k_condense<1, 0, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<2, 0, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<3, 0, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<4, 0, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<8, 0, 1, MODE_COLUMNS>),
      reinterpret_cast<const void*>(&k_condense<1, 0, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<2, 0, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<3, 0, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<4, 0, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_condense<8, 0, 1, MODE_RECOVER>),
      reinterpret_cast<const void*>(&k_gx_solve<1, 0, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<2, 0, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<3, 0, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<4, 0, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<8, 0, 0>),
      reinterpret_cast<const void*>(&k_gx_solve<1, 0, 1>),
      reinterpret_cast<const void*>(&k_gx_solve<2, 0, 1>),
      reinterpret_cast<const void*>(&k_gx_solve<3, 0, 1>),
      reinterpret_cast<const void*>(&k_gx_solve<4, 0, 1>),
      reinterpret_cast<const void*>(&k_gx_solve<8, 0, 1>)};
  for (const void* f : fns)
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  const void* bfns[] = {
      reinterpret_cast<const void*>(&k_condense_b<1, 2>),
      reinterpret_cast<const void*>(&k_condense_b<1, 2, kCondWaves>),
      reinterpret_cast<const void*>(&k_condense_b<1, 1, kCondWaves>),
      reinterpret_cast<const void*>(&k_condense_b<1, 2, kCondWavesWide>),
      reinterpret_cast<const void*>(&k_condense_b<1, 1, kCondWavesWide>),
      reinterpret_cast<const void*>(&k_condense_b<1, 1, kCondWavesPair>),
      reinterpret_cast<const void*>(&k_condense_b<1, 2, kCondWavesPair>),
      reinterpret_cast<const void*>(&k_condense_b<1, 1>),
      reinterpret_cast<const void*>(&k_condense_b<2, 1>),
      reinterpret_cast<const void*>(&k_condense_b<3, 1>),
      reinterpret_cast<const void*>(&k_condense_b<4, 1>),
      reinterpret_cast<const void*>(&k_condense_b<8, 1>),
      reinterpret_cast<const void*>(&k_condense_b<1, 0>),
      reinterpret_cast<const void*>(&k_condense_b<2, 0>),
      reinterpret_cast<const void*>(&k_condense_b<3, 0>),
      reinterpret_cast<const void*>(&k_condense_b<4, 0>),
      reinterpret_cast<const void*>(&k_condense_b<8, 0>),
      reinterpret_cast<const void*>(&k_refactor_wave_b),
      reinterpret_cast<const void*>(&k_refactor_level_staged),
      reinterpret_cast<const void*>(&k_refactor_level_staged_b),
      reinterpret_cast<const void*>(&k_refactor_b)};
  for (const void* f : bfns)
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  for (const void* f : gfns)
    (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, max_lds_bytes());
  (void)hipGetLastError();
}

int device_cus() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
    return 256;
  return v;
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
                             const double* sig_s, double* sig_s_keep, hipStream_t st) {
  const int grid = cdiv(d.nnz_k, kBlock);
  hipLaunchKernelGGL(k_assemble_k, dim3(grid > 0 ? grid : 1), dim3(kBlock), 0, st, d, sig_x,
                     sig_u, sig_s, sig_s_keep);
  return hipGetLastError();
}

hipError_t launch_refactor(const DevNet& d, hipStream_t st) {
  hipLaunchKernelGGL(k_fill_int, dim3(1), dim3(64), 0, st, d.status + 2, 2, 0);
  if (d.rw_ok) {
    for (int lev = 1; lev <= d.rw_split; ++lev)
      hipLaunchKernelGGL(k_refactor_level, dim3(d.rw_split_grid, kRwWaves), dim3(64), 0, st, d,
                         lev);
    hipLaunchKernelGGL(k_refactor_wave, dim3(32), dim3(kRwWaves * 64),
                       (size_t)(d.rw_nnz_u + 1 + d.nx) * sizeof(double) +
                           (size_t)kRwWaves * d.rw_nlev * sizeof(int), st, d, d.rw_split);
  }
  else if (d.rf_per_level)
    for (int lev = 0; lev < d.rf_nlev; ++lev)
      hipLaunchKernelGGL(k_refactor_level_staged, dim3(d.rf_level_grid), dim3(kRefThreads),
                         (size_t)d.rf_lds_doubles * sizeof(double), st, d, lev);
  else
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

hipError_t launch_recover(const DevNet& d, int width, bool lds, const double* pu,
                          const double* r, double* p, hipStream_t st) {
  if (lds)
    return dispatch_width<true>(d, 0, 1, width, MODE_RECOVER, r, pu, nullptr, 0, nullptr, p, st);
  return dispatch_width<false>(d, 0, 1, width, MODE_RECOVER, r, pu, nullptr, 0, nullptr, p, st);
}

template <int W, int PM, int TRANS>
hipError_t launch_gx_solve_t(const DevNet& d, const double* b, double* x, double scale,
                             int accumulate, hipStream_t st) {
  hipLaunchKernelGGL((k_gx_solve<W, PM, TRANS>), dim3(1), dim3(kCondThreads),
                     condense_lds_bytes(d, W, PM != 0, 1), st, d, b, x, scale, accumulate);
  return hipGetLastError();
}

template <bool LDS, int TRANS>
hipError_t gx_solve_width(const DevNet& d, int width, const double* b, double* x, double scale,
                          int accumulate, hipStream_t st) {
  if (LDS && d.meta_global) {
    if (width != 1) return hipErrorInvalidValue;
    return launch_gx_solve_t<1, 2, TRANS>(d, b, x, scale, accumulate, st);
  }
  switch (width) {
    case 1: return launch_gx_solve_t<1, LDS, TRANS>(d, b, x, scale, accumulate, st);
    case 2: return launch_gx_solve_t<2, LDS, TRANS>(d, b, x, scale, accumulate, st);
    case 3: return launch_gx_solve_t<3, LDS, TRANS>(d, b, x, scale, accumulate, st);
    case 4: return launch_gx_solve_t<4, LDS, TRANS>(d, b, x, scale, accumulate, st);
    case 8: return launch_gx_solve_t<8, LDS, TRANS>(d, b, x, scale, accumulate, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_gx_solve(const DevNet& d, int width, bool lds, bool transpose, const double* b,
                           double* x, double scale, bool accumulate, hipStream_t st) {
  const int acc = accumulate ? 1 : 0;
  if (lds)
    return transpose ? gx_solve_width<true, 1>(d, width, b, x, scale, acc, st)
                     : gx_solve_width<true, 0>(d, width, b, x, scale, acc, st);
  return transpose ? gx_solve_width<false, 1>(d, width, b, x, scale, acc, st)
                   : gx_solve_width<false, 0>(d, width, b, x, scale, acc, st);
}

hipError_t launch_recover_stored(const DevNet& d, double* p, hipStream_t st) {
  hipLaunchKernelGGL(k_recover_partial, dim3(cdiv(d.nx, kBlock), kRecChunks), dim3(kBlock), 0, st,
                     d, (const double*)p);
  hipLaunchKernelGGL(k_recover_finish, dim3(cdiv(d.nx > d.nu ? d.nx : d.nu, kBlock)), dim3(kBlock),
                     0, st, d, p);
  return hipGetLastError();
}

hipError_t launch_finish_step(const DevNet& d, const double* r, const double* sig_s, double* p,
                              int* hstat, hipStream_t st) {
  const int grid = cdiv(d.m, kBlock);
  hipLaunchKernelGGL(k_finish_step, dim3(grid > 0 ? grid : 1), dim3(kBlock), 0, st, d, r, sig_s, p,
                     hstat);
  return hipGetLastError();
}

hipError_t launch_symmetrize(double* K, long ldk, int n, double* copy, hipStream_t st) {
  hipLaunchKernelGGL(k_symmetrize, dim3(cdiv(n, 16), cdiv(n, 16)), dim3(16, 16), 0, st, K, ldk, n,
                     copy);
  return hipGetLastError();
}

hipError_t launch_batch_condense(const DevNet* nets, const BatchArg* args, const int2* tiles,
                                 const BatchShape& sh, hipStream_t st) {
  const int B = sh.count;
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval_lines_b, dim3(cdiv(sh.max_lines, kBlock), 1, B), dim3(kBlock), 0, st,
                     nets, args, 1);
  hipLaunchKernelGGL(k_gather_b, dim3(cdiv(sh.max_dst, kBlock), 1, B), dim3(kBlock), 0, st, nets);
  hipLaunchKernelGGL(k_copy_b, dim3(cdiv(sh.max_m, kBlock), 1, B), dim3(kBlock), 0, st, args, 0);
  hipLaunchKernelGGL(k_assemble_k_b, dim3(cdiv(sh.max_nnz_k, kBlock), 1, B), dim3(kBlock), 0, st,
                     nets, args);
  hipLaunchKernelGGL(k_rtilde_b, dim3(cdiv(sh.max_nw, kBlock), 1, B), dim3(kBlock), 0, st, nets,
                     args);
  hipLaunchKernelGGL(k_clear_status_b, dim3(1, 1, B), dim3(64), 0, st, nets, 2, 2);
  if (sh.any_wave) {
    for (int lev = 1; lev <= sh.max_split; ++lev)
      hipLaunchKernelGGL(k_refactor_level_b, dim3(sh.max_split_grid, kRwWaves, B), dim3(64), 0, st,
                         nets, lev);
    hipLaunchKernelGGL(k_refactor_wave_b, dim3(1, 1, B), dim3(kRwWaves * 64), sh.lds_wave, st,
                       nets);
  }
  if (sh.any_staged)
    hipLaunchKernelGGL(k_refactor_b, dim3(1, 1, B), dim3(kRefThreads), sh.lds_staged, st, nets);
  for (int lev = 0; lev < sh.max_staged_levels; ++lev)
    hipLaunchKernelGGL(k_refactor_level_staged_b, dim3(sh.max_staged_grid, 1, B), dim3(kRefThreads),
                       sh.lds_staged, st, nets, lev);
  hipLaunchKernelGGL(k_transcribe_b, dim3(64, 1, B), dim3(kBlock), 0, st, nets);
  // one condensation launch per class of members (panel width and placement)
  for (const CondClass& c : sh.cls) {
    if (c.ntiles == 0) continue;
    const int2* ct = tiles + c.tile0;
    const int W = c.width;
#define RH_BATCH_COND(WW, LL)                                                                   \
  hipLaunchKernelGGL((k_condense_b<WW, LL>), dim3(c.ntiles), dim3(64), c.lds_bytes, st, nets, args, \
                     ct)
#define RH_BATCH_COND_WAVES(LL, NWV)                                                            \
  hipLaunchKernelGGL((k_condense_b<1, LL, NWV>), dim3(c.ntiles), dim3(64 * NWV), c.lds_bytes, st, \
                     nets, args, ct)
    const int nwv = c.lds ? c.nw : 1;
    if (nwv != 1 && nwv != kCondWavesPair && nwv != kCondWaves && nwv != kCondWavesWide)
      return hipErrorInvalidValue;
    if (nwv > 1 && W != 1) return hipErrorInvalidValue;
    if (W != 1 && W != 2 && W != 3 && W != 4 && W != 8) return hipErrorInvalidValue;
    if (c.lds && c.meta_global) {
      if (W != 1) return hipErrorInvalidValue;
      if (nwv == kCondWavesPair) RH_BATCH_COND_WAVES(2, kCondWavesPair);
      else if (nwv == kCondWavesWide) RH_BATCH_COND_WAVES(2, kCondWavesWide);
      else if (nwv == kCondWaves) RH_BATCH_COND_WAVES(2, kCondWaves);
      else RH_BATCH_COND(1, 2);
    } else if (c.lds) {
      if (nwv == kCondWavesPair) RH_BATCH_COND_WAVES(1, kCondWavesPair);
      else if (nwv == kCondWavesWide) RH_BATCH_COND_WAVES(1, kCondWavesWide);
      else if (nwv == kCondWaves) RH_BATCH_COND_WAVES(1, kCondWaves);
      else if (W == 1) RH_BATCH_COND(1, 1);
      else if (W == 2) RH_BATCH_COND(2, 1);
      else if (W == 3) RH_BATCH_COND(3, 1);
      else if (W == 4) RH_BATCH_COND(4, 1);
      else RH_BATCH_COND(8, 1);
    } else {
      if (W == 1) RH_BATCH_COND(1, 0);
      else if (W == 2) RH_BATCH_COND(2, 0);
      else if (W == 3) RH_BATCH_COND(3, 0);
      else if (W == 4) RH_BATCH_COND(4, 0);
      else RH_BATCH_COND(8, 0);
    }
#undef RH_BATCH_COND
#undef RH_BATCH_COND_WAVES
  }
  hipLaunchKernelGGL(k_symmetrize_b, dim3(cdiv(sh.max_nu, 16), cdiv(sh.max_nu, 16), B),
                     dim3(16, 16), 0, st, args);
  return hipGetLastError();
}

hipError_t launch_batch_solve(const DevNet* nets, const BatchArg* args, const BatchShape& sh,
                              hipStream_t st) {
  const int B = sh.count;
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_copy_b, dim3(cdiv(sh.max_nu, kBlock), 1, B), dim3(kBlock), 0, st, args, 1);
  hipLaunchKernelGGL(k_clear_status_b, dim3(1, 1, B), dim3(64), 0, st, nets, 0, 2);
  {
    const hipError_t e = launch_batch_cholesky(args, sh.orders, st);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_recover_partial_b, dim3(cdiv(sh.max_nx, kBlock), kRecChunks, B),
                     dim3(kBlock), 0, st, nets, args);
  hipLaunchKernelGGL(k_recover_finish_b,
                     dim3(cdiv(sh.max_nx > sh.max_nu ? sh.max_nx : sh.max_nu, kBlock), 1, B),
                     dim3(kBlock), 0, st, nets, args);
  hipLaunchKernelGGL(k_finish_step_b, dim3(cdiv(sh.max_m, kBlock), 1, B), dim3(kBlock), 0, st,
                     nets, args);
  return hipGetLastError();
}

hipError_t launch_batch_status(const DevNet* nets, int count, int* out, hipStream_t st) {
  if (count > 0) hipLaunchKernelGGL(k_gather_status_b, dim3(1, 1, count), dim3(64), 0, st, nets, out);
  return hipGetLastError();
}

hipError_t launch_batch_ipm_eval(const DevNet* nets, const BatchArg* args, const IpmDev* ipms,
                                 const double* sc, const BatchShape& sh, int trial,
                                 hipStream_t st) {
  const int B = sh.count;
  if (B == 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval_lines_b, dim3(cdiv(sh.max_lines, kBlock), 1, B), dim3(kBlock), 0, st,
                     nets, args, trial ? 0 : 1);
  hipLaunchKernelGGL(k_gather_b, dim3(cdiv(sh.max_dst, kBlock), 1, B), dim3(kBlock), 0, st, nets);
  hipLaunchKernelGGL(k_objective_b, dim3(1, 1, B), dim3(kBlock), 0, st, nets, ipms, sc, trial);
  return hipGetLastError();
}

hipError_t launch_eval_objective(const DevNet& d, const double* u, double* f, hipStream_t st) {
  hipLaunchKernelGGL(k_objective, dim3(1), dim3(kBlock), 0, st, d, u, d.c2, d.c1, d.c0, d.pg_u, f);
  return hipGetLastError();
}

}  // namespace rh
