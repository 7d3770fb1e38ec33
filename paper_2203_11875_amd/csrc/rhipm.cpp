// C ABI of the condensation hot path (declarations and contracts in rhipm.h).
#include "rhipm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <memory>
#include <new>
#include <vector>

#include "analysis.hpp"
#include "device.hpp"

struct rh_symbolic {
  rh::Symbolic s;
};

// Per-phase device timers (hipEvent pairs recorded on the handle's stream).
struct PhaseTimer {
  static constexpr int kPool = 128;
  std::vector<hipEvent_t> ev;   // 2 * kPool
  int used = 0;
  double ms = 0.0;
  long calls = 0;
};

struct rh_net {
  rh::Symbolic s;
  bool profiling = false;
  PhaseTimer timers[RH_NPHASES];
  rh::DevNet d{};
  hipStream_t stream = nullptr;
  std::vector<void*> allocs;
  int width = 2;
  bool lds = true;
  bool condensed = false;
  bool rhs_cols = false;     // the last condensation stored the right-hand-side column
  double* sig_s = nullptr;   // copy of Sigma_s from the last condensation
  double* bwork = nullptr;   // Cholesky right-hand-side work copy
  double* cinv = nullptr;    // 32 x 32 diagonal blocks of the Cholesky factor: inverses, then factors
  double* lrow = nullptr;    // the Cholesky factor by row blocks (backward substitution)
  int* status = nullptr;
  long long* trace = nullptr;
  size_t panel_cap = 0;
};

namespace {

void drain(PhaseTimer& t) {
  for (int k = 0; k < t.used; ++k) {
    float ms = 0.f;
    if (hipEventSynchronize(t.ev[2 * k + 1]) == hipSuccess &&
        hipEventElapsedTime(&ms, t.ev[2 * k], t.ev[2 * k + 1]) == hipSuccess) {
      t.ms += ms;
      t.calls += 1;
    }
  }
  t.used = 0;
}

// RAII: records the start event on construction and the stop event on
// destruction when profiling is on.
struct PhaseScope {
  rh_net* n;
  int ph;
  PhaseScope(rh_net* net, int phase) : n(net), ph(phase) {
    if (!n->profiling) return;
    PhaseTimer& t = n->timers[ph];
    if (t.ev.empty()) {
      t.ev.resize(2 * PhaseTimer::kPool);
      for (auto& e : t.ev) (void)hipEventCreate(&e);
    }
    if (t.used == PhaseTimer::kPool) drain(t);
    (void)hipEventRecord(t.ev[2 * t.used], n->stream);
  }
  ~PhaseScope() {
    if (!n->profiling) return;
    PhaseTimer& t = n->timers[ph];
    (void)hipEventRecord(t.ev[2 * t.used + 1], n->stream);
    t.used += 1;
  }
};

template <typename T>
rh_status upload(rh_net* n, const std::vector<T>& v, const T** out) {
  void* p = nullptr;
  size_t bytes = std::max<size_t>(1, v.size()) * sizeof(T);
  if (hipMalloc(&p, bytes) != hipSuccess) return RH_ERR_OOM;
  n->allocs.push_back(p);
  if (!v.empty() && hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return RH_ERR_HIP;
  *out = static_cast<const T*>(p);
  return RH_OK;
}

template <typename T>
rh_status alloc(rh_net* n, size_t count, T** out) {
  void* p = nullptr;
  if (hipMalloc(&p, std::max<size_t>(1, count) * sizeof(T)) != hipSuccess) return RH_ERR_OOM;
  n->allocs.push_back(p);
  *out = static_cast<T*>(p);
  return RH_OK;
}

#define RH_TRY(expr)               \
  do {                             \
    rh_status _st = (expr);        \
    if (_st != RH_OK) return _st;  \
  } while (0)
#define RH_HIP(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return RH_ERR_HIP;  \
  } while (0)

rh_status upload_sweep(rh_net* n, const rh::Sweep& s, rh::DevSweep& d) {
  d.nlev = s.nlev;
  d.nnz = int(s.col.size());
  RH_TRY(upload(n, s.lev_ptr, &d.lev_ptr));
  RH_TRY(upload(n, s.rows, &d.rows));
  RH_TRY(upload(n, s.ptr, &d.ptr));
  RH_TRY(upload(n, s.col, &d.col));
  RH_TRY(upload(n, s.src, &d.src));
  RH_TRY(upload(n, s.lev_lanes, &d.lev_lanes));
  RH_TRY(upload(n, s.lev_base, &d.lev_base));
  RH_TRY(upload(n, s.lev_len, &d.lev_len));
  RH_TRY(upload(n, s.ell_col, &d.ell_col));
  RH_TRY(upload(n, s.ell_src, &d.ell_src));
  RH_TRY(alloc(n, s.ell_col.size(), &d.ell_val));
  d.ell_n = int(s.ell_col.size());
  RH_TRY(alloc(n, s.col.size(), &d.val));
  d.unit = s.has_diag ? 0 : 1;
  if (s.has_diag) {
    RH_TRY(upload(n, s.diag_src, &d.diag_src));
    RH_TRY(alloc(n, s.diag_src.size(), &d.dinv));
  } else {
    d.diag_src = nullptr;
    const double* ones;
    RH_TRY(upload(n, std::vector<double>(s.rows.size(), 1.0), &ones));
    d.dinv = const_cast<double*>(ones);
  }
  return RH_OK;
}

void fill_info(const rh::Symbolic& s, rh_info* info) {
  std::memset(info, 0, sizeof(*info));
  info->nx = s.nx;
  info->nu = s.nu;
  info->m = s.m;
  info->nb = s.nb;
  info->nl = s.nl;
  info->ng = s.ng;
  info->nnz_gx = long(s.gx_col.size());
  info->nnz_lu = long(s.lu_col.size());
  info->nnz_gu = long(s.gu_col.size());
  info->nnz_a = long(s.a_col.size());
  info->nnz_k = long(s.k_col.size());
  info->levels_lower = s.sl.nlev;
  info->levels_upper = s.su.nlev;
  info->refactor_ops = s.refactor_ops;
  info->max_lu_row = s.max_row;
  info->max_row_ops = s.max_row_ops;
  info->refactor_kernel = s.rw_ok ? 0 : 1;
}

void copy_maps(const rh::Symbolic& s, int32_t* x_kind, int32_t* x_bus, int32_t* u_kind,
               int32_t* u_ref) {
  if (x_kind) std::copy(s.x_kind.begin(), s.x_kind.end(), x_kind);
  if (x_bus) std::copy(s.x_bus.begin(), s.x_bus.end(), x_bus);
  if (u_kind) std::copy(s.u_kind.begin(), s.u_kind.end(), u_kind);
  if (u_ref) std::copy(s.u_ref.begin(), s.u_ref.end(), u_ref);
}

rh_status build_device(rh_net* n, const rh_network_desc& desc, const rh_options* opts) {
  const rh::Symbolic& s = n->s;
  rh::DevNet& d = n->d;
  d.nb = s.nb; d.nl = s.nl; d.ng = s.ng; d.nx = s.nx; d.nu = s.nu; d.m = s.m; d.nw = s.nw;
  d.nlim = s.nlim; d.ref = s.ref; d.ref_gen = s.ref_gen;
  d.base = s.base;
  d.c2_ref = desc.c2[s.ref_gen];
  d.c1_ref = desc.c1[s.ref_gen];
  d.cost_rank1 = s.cost_rank1;
  RH_TRY(upload(n, std::vector<double>(desc.c2, desc.c2 + s.ng), &d.c2));
  RH_TRY(upload(n, std::vector<double>(desc.c1, desc.c1 + s.ng), &d.c1));
  RH_TRY(upload(n, std::vector<double>(desc.c0, desc.c0 + s.ng), &d.c0));
  RH_TRY(upload(n, s.pg_u, &d.pg_u));
  RH_TRY(upload(n, s.lf, &d.lf));
  RH_TRY(upload(n, s.lt, &d.lt));
  RH_TRY(upload(n, s.gff, &d.gff));
  RH_TRY(upload(n, s.bff, &d.bff));
  RH_TRY(upload(n, s.gft, &d.gft));
  RH_TRY(upload(n, s.bft, &d.bft));
  RH_TRY(upload(n, s.th_nat, &d.th_nat));
  RH_TRY(upload(n, s.vmx_nat, &d.vmx_nat));
  RH_TRY(upload(n, s.vmu, &d.vmu));
  RH_TRY(upload(n, s.line_w, &d.line_w));
  RH_TRY(upload(n, s.line_wsrc, &d.line_wsrc));
  RH_TRY(upload(n, s.ref_lines, &d.ref_lines));
  RH_TRY(upload(n, s.ref_ends, &d.ref_ends));
  d.n_ref_lines = int(s.ref_lines.size());
  RH_TRY(upload(n, s.perm, &d.perm));
  RH_TRY(upload(n, s.iperm, &d.iperm));
  d.nnz_lu = int(s.lu_col.size());
  d.max_row = s.max_row;
  RH_TRY(upload(n, s.lu_ptr, &d.lu_ptr));
  RH_TRY(upload(n, s.lu_col, &d.lu_col));
  RH_TRY(upload(n, s.lu_diag, &d.lu_diag));
  RH_TRY(upload(n, s.rf_kptr, &d.rf_kptr));
  RH_TRY(upload(n, s.rf_op_src, &d.rf_src));
  RH_TRY(upload(n, s.rf_op_dst, &d.rf_dst));
  RH_TRY(upload(n, s.rf_piv, &d.rf_piv));
  RH_TRY(upload(n, s.rf_dst_local, &d.rf_dst_local));
  d.max_row_ops = s.max_row_ops;
  d.max_row_lower = s.max_row_lower;
  RH_TRY(upload_sweep(n, s.sl, d.sl));
  RH_TRY(upload_sweep(n, s.su, d.su));
  RH_TRY(upload_sweep(n, s.sut, d.sut));
  RH_TRY(upload_sweep(n, s.slt, d.slt));
  d.rf_rows = d.sl.rows;
  d.rf_lev_ptr = d.sl.lev_ptr;
  d.rf_nlev = d.sl.nlev;
  d.nnz_gu = int(s.gu_col.size());
  d.nnz_a = int(s.a_col.size());
  d.nnz_k = int(s.k_col.size());
  RH_TRY(upload(n, s.gu_ptr, &d.gu_ptr));
  RH_TRY(upload(n, s.gu_col, &d.gu_col));
  RH_TRY(upload(n, s.gucsc_ptr, &d.gucsc_ptr));
  RH_TRY(upload(n, s.gucsc_row, &d.gucsc_row));
  RH_TRY(upload(n, s.gucsc_from_csr, &d.gucsc_from));
  RH_TRY(upload(n, s.a_ptr, &d.a_ptr));
  RH_TRY(upload(n, s.a_col, &d.a_col));
  RH_TRY(upload(n, s.acsc_ptr, &d.acsc_ptr));
  RH_TRY(upload(n, s.acsc_row, &d.acsc_row));
  RH_TRY(upload(n, s.acsc_from_csr, &d.acsc_from));
  RH_TRY(upload(n, s.k_ptr, &d.k_ptr));
  RH_TRY(upload(n, s.k_col, &d.k_col));
  RH_TRY(upload(n, s.kg.hl_ptr, &d.kg_hl_ptr));
  RH_TRY(upload(n, s.kg.hl_idx, &d.kg_hl_idx));
  RH_TRY(upload(n, s.kg.ata_ptr, &d.kg_ata_ptr));
  RH_TRY(upload(n, s.kg.ata_a1, &d.kg_a1));
  RH_TRY(upload(n, s.kg.ata_a2, &d.kg_a2));
  RH_TRY(upload(n, s.kg.ata_row, &d.kg_row));
  RH_TRY(upload(n, s.kg.diag_var, &d.kg_diag));
  RH_TRY(upload(n, s.sig_map, &d.sig_map));
  RH_TRY(upload(n, s.kb_base, &d.kb_base));
  RH_TRY(upload(n, s.kb_len, &d.kb_len));
  RH_TRY(upload(n, s.kell_col, &d.kell_col));
  RH_TRY(upload(n, s.kell_pos, &d.kell_pos));
  RH_TRY(alloc(n, s.kell_col.size(), &d.kell_val));
  d.kell_n = int(s.kell_col.size());
  d.kb_n = int(s.kb_base.size());
  d.rw_ok = s.rw_ok ? 1 : 0;
  d.rw_nnz_u = s.rw_nnz_u;
  d.rw_nlev = s.sl.nlev;
  d.rw_wbeg = d.rw_levend = d.rw_rec = d.rw_lane = d.rw_ustart = nullptr;
  d.rw_ntask = 0;
  d.rw_lane_pad = 0;
  if (s.rw_ok) {
    d.rw_ntask = int(s.rw_rec.size()) / rh::kRwRec - 1;
    d.rw_lane_pad = int(s.rw_lane.size()) - 64;
    RH_TRY(upload(n, s.rw_wbeg, &d.rw_wbeg));
    RH_TRY(upload(n, s.rw_levend, &d.rw_levend));
    RH_TRY(upload(n, s.rw_rec, &d.rw_rec));
    RH_TRY(upload(n, s.rw_lane, &d.rw_lane));
    RH_TRY(upload(n, s.rw_ustart, &d.rw_ustart));
  }
  RH_TRY(upload(n, s.rf_lmeta, &d.rf_lmeta));
  d.rf_lds_doubles = s.rf_lds_doubles;
  RH_TRY(upload(n, s.k_cdiag, &d.k_cdiag));
  d.d_total = s.d_total; d.d_lu = s.d_lu; d.d_gu = s.d_gu; d.d_a = s.d_a; d.d_g = s.d_g;
  d.d_h = s.d_h; d.src_u = s.src_u; d.src_total = s.src_total;
  RH_TRY(upload(n, s.eg.ptr, &d.eg_ptr));
  RH_TRY(upload(n, s.eg.idx, &d.eg_idx));
  RH_TRY(upload(n, s.eg.coef, &d.eg_coef));
  RH_TRY(upload(n, s.eg.cst, &d.eg_cst));
  // workspaces
  {
    std::vector<double> src(s.src_total, 0.0);
    std::copy(desc.pd, desc.pd + s.nb, src.begin() + s.src_u + s.nu);
    std::copy(desc.qd, desc.qd + s.nb, src.begin() + s.src_u + s.nu + s.nb);
    const double* p;
    RH_TRY(upload(n, src, &p));
    d.src = const_cast<double*>(p);
  }
  RH_TRY(alloc(n, s.d_total, &d.dst));
  RH_TRY(alloc(n, size_t(rh::HL_STRIDE) * s.nl, &d.hl));
  RH_TRY(alloc(n, s.k_col.size(), &d.kval));
  RH_TRY(alloc(n, s.nw, &d.rt));
  RH_TRY(alloc(n, s.nw, &d.pw));
  RH_TRY(alloc(n, s.nu, &d.vtmp));
  RH_TRY(alloc(n, s.nx, &d.rinv));
  RH_TRY(alloc(n, size_t(s.nx) * (s.nu + 1), &d.zcols));
  RH_TRY(alloc(n, size_t(s.nx) * (s.nu + 1), &d.psicols));
  RH_TRY(alloc(n, size_t(2) * 8 * s.nx, &d.rpart));
  {
    std::vector<int> info;
    for (int q = 0; q < s.nx; ++q) {
      const int i = s.sl.rows[q];
      const int rp0 = s.lu_ptr[i], rd = s.lu_diag[i];
      info.insert(info.end(), {i, rp0, s.lu_ptr[i + 1], rd, s.rf_kptr[rp0],
                               s.rf_kptr[rd] - s.rf_kptr[rp0], 0, 0});
    }
    RH_TRY(upload(n, info, &d.rf_info));
  }
  RH_TRY(alloc(n, s.m, &n->sig_s));
  RH_TRY(alloc(n, s.nu, &n->bwork));
  RH_TRY(alloc(n, 2 * size_t((s.nu + 31) / 32) * 32 * 32, &n->cinv));
  RH_TRY(alloc(n, size_t((s.nu + 31) / 32 * 32) * size_t((s.nu + 31) / 32 * 32), &n->lrow));
  RH_TRY(alloc(n, 8, &n->status));
  RH_TRY(alloc(n, 256, &n->trace));
  RH_HIP(hipMemset(n->trace, 0, 256 * sizeof(long long)));
  d.trace = nullptr;
  d.status = n->status;
  RH_HIP(hipMemset(n->status, 0, 8 * sizeof(int)));
  // launch shape of the condensation
  const size_t col_bytes = size_t(s.nw) * sizeof(double);   // one LDS panel column
  const size_t lds_max = size_t(rh::max_lds_bytes());
  const size_t meta = rh::condense_meta_bytes(d);
  int want = opts && opts->panel_width > 0 ? opts->panel_width : 1;
  if (want != 1 && want != 2 && want != 3 && want != 4 && want != 8) return RH_ERR_ARG;
  bool lds = (!opts || opts->lds_panel != 0) && int(s.kb_base.size()) <= rh::kMaxRowBlocks;
  if (lds && col_bytes * want + meta > lds_max) {
    // keep the panel in LDS with a narrower tile if possible
    int w = want;
    while (w > 1 && col_bytes * w + meta > lds_max) w = (w == 8 ? 4 : w - 1);
    if (col_bytes * w + meta <= lds_max) want = w; else lds = false;
  }
  if (meta > lds_max) return RH_ERR_ARG;
  n->width = want;
  n->lds = lds;
  rh::prepare_lds_kernels(lds ? col_bytes * want + meta : meta);
  d.panel = nullptr;
  d.panel_doubles = 0;
  if (!lds) {
    const size_t nblk = (size_t(s.nu) + 1 + want - 1) / want;
    d.panel_doubles = nblk * 2 * size_t(s.nw) * want;
    RH_TRY(alloc(n, d.panel_doubles, &d.panel));
  }
  if (size_t(s.rf_lds_doubles) * sizeof(double) > lds_max) return RH_ERR_ARG;
  RH_HIP(hipDeviceSynchronize());
  return RH_OK;
}

}  // namespace

extern "C" {

const char* rh_status_str(rh_status s) {
  switch (s) {
    case RH_OK: return "ok";
    case RH_NOT_POSDEF: return "condensed matrix not positive definite";
    case RH_SMALL_PIVOT: return "small pivot in the refactorisation of G_x";
    case RH_NOT_CONVERGED: return "not converged";
    case RH_ERR_ARG: return "invalid argument";
    case RH_ERR_HIP: return "HIP runtime error";
    case RH_ERR_OOM: return "out of memory";
    case RH_ERR_SINGULAR: return "structurally singular state Jacobian";
    case RH_ERR_STATE: return "invalid call order";
  }
  return "unknown status";
}

rh_status rh_analyze_network(const rh_network_desc* desc, const rh_options* opts,
                             rh_symbolic** out) {
  if (!desc || !out) return RH_ERR_ARG;
  *out = nullptr;
  auto* sym = new (std::nothrow) rh_symbolic();
  if (!sym) return RH_ERR_OOM;
  rh_status st = rh::analyze(*desc, opts, sym->s);
  if (st != RH_OK) {
    delete sym;
    return st;
  }
  *out = sym;
  return RH_OK;
}

void rh_destroy_symbolic(rh_symbolic* sym) { delete sym; }

rh_status rh_symbolic_info(const rh_symbolic* sym, rh_info* info) {
  if (!sym || !info) return RH_ERR_ARG;
  fill_info(sym->s, info);
  return RH_OK;
}

rh_status rh_symbolic_index_maps(const rh_symbolic* sym, int32_t* x_kind, int32_t* x_bus,
                                 int32_t* u_kind, int32_t* u_ref) {
  if (!sym) return RH_ERR_ARG;
  copy_maps(sym->s, x_kind, x_bus, u_kind, u_ref);
  return RH_OK;
}

rh_status rh_symbolic_gx_pattern(const rh_symbolic* sym, int32_t* rowptr, int32_t* col,
                                 int32_t* perm) {
  if (!sym) return RH_ERR_ARG;
  const auto& s = sym->s;
  if (rowptr) std::copy(s.gx_ptr.begin(), s.gx_ptr.end(), rowptr);
  if (col) std::copy(s.gx_col.begin(), s.gx_col.end(), col);
  if (perm) std::copy(s.perm.begin(), s.perm.end(), perm);
  return RH_OK;
}

rh_status rh_symbolic_host_solve(const rh_symbolic* sym, const double* gx_values,
                                 const double* b, double* z, int32_t transpose) {
  if (!sym || !gx_values || !b || !z) return RH_ERR_ARG;
  return rh::host_solve(sym->s, gx_values, b, z, transpose != 0);
}

rh_status rh_symbolic_check_levels(const rh_symbolic* sym) {
  if (!sym) return RH_ERR_ARG;
  return rh::check_levels(sym->s);
}

rh_status rh_init_network(const rh_network_desc* desc, const rh_options* opts, void* hip_stream,
                          rh_net** out) {
  if (!desc || !out) return RH_ERR_ARG;
  *out = nullptr;
  auto* n = new (std::nothrow) rh_net();
  if (!n) return RH_ERR_OOM;
  n->stream = static_cast<hipStream_t>(hip_stream);
  rh_status st = rh::analyze(*desc, opts, n->s);
  if (st == RH_OK) st = build_device(n, *desc, opts);
  if (st != RH_OK) {
    rh_destroy_network(n);
    return st;
  }
  *out = n;
  return RH_OK;
}

void rh_destroy_network(rh_net* n) {
  if (!n) return;
  if (n->stream) (void)hipStreamSynchronize(n->stream);
  else (void)hipDeviceSynchronize();
  for (auto& t : n->timers)
    for (auto& e : t.ev) (void)hipEventDestroy(e);
  for (void* p : n->allocs) (void)hipFree(p);
  delete n;
}

rh_status rh_get_info(const rh_net* n, rh_info* info) {
  if (!n || !info) return RH_ERR_ARG;
  fill_info(n->s, info);
  info->panel_width = n->width;
  info->lds_panel = n->lds ? 1 : 0;
  return RH_OK;
}

rh_status rh_get_dims(const rh_net* n, int64_t* nx, int64_t* nu, int64_t* m) {
  if (!n) return RH_ERR_ARG;
  if (nx) *nx = n->s.nx;
  if (nu) *nu = n->s.nu;
  if (m) *m = n->s.m;
  return RH_OK;
}

rh_status rh_get_index_maps(const rh_net* n, int32_t* x_kind, int32_t* x_bus, int32_t* u_kind,
                            int32_t* u_ref) {
  if (!n) return RH_ERR_ARG;
  copy_maps(n->s, x_kind, x_bus, u_kind, u_ref);
  return RH_OK;
}

rh_status rh_set_loads(rh_net* n, const double* pd, const double* qd) {
  if (!n || !pd || !qd) return RH_ERR_ARG;
  double* base = n->d.src + n->s.src_u + n->s.nu;
  RH_HIP(hipMemcpyAsync(base, pd, sizeof(double) * n->s.nb, hipMemcpyDeviceToDevice, n->stream));
  RH_HIP(hipMemcpyAsync(base + n->s.nb, qd, sizeof(double) * n->s.nb, hipMemcpyDeviceToDevice,
                        n->stream));
  return RH_OK;
}

rh_status rh_eval_residual(rh_net* n, const double* x, const double* u, double* g, double* h,
                           double* f) {
  if (!n || !x || !u) return RH_ERR_ARG;
  const auto& d = n->d;
  RH_HIP(rh::launch_eval(d, x, u, nullptr, nullptr, false, n->stream));
  if (g)
    RH_HIP(hipMemcpyAsync(g, d.dst + d.d_g, sizeof(double) * d.nx, hipMemcpyDeviceToDevice,
                          n->stream));
  if (h)
    RH_HIP(hipMemcpyAsync(h, d.dst + d.d_h, sizeof(double) * d.m, hipMemcpyDeviceToDevice,
                          n->stream));
  if (f) RH_HIP(rh::launch_eval_objective(d, u, f, n->stream));
  return RH_OK;
}

rh_status rh_condense_reduced_hessian(rh_net* n, const double* x, const double* u,
                                      const double* lam, const double* y, const double* sig_x,
                                      const double* sig_u, const double* sig_s, const double* r,
                                      double* K, int64_t ldk, double* rhs) {
  if (!n || !x || !u || !lam || !y || !sig_x || !sig_u || !sig_s || !K) return RH_ERR_ARG;
  if (ldk < n->s.nu || (r && !rhs) || (rhs && !r)) return RH_ERR_ARG;
  const auto& d = n->d;
  hipStream_t st = n->stream;
  n->condensed = false;
  RH_HIP(hipMemcpyAsync(n->sig_s, sig_s, sizeof(double) * d.m, hipMemcpyDeviceToDevice, st));
  {
    PhaseScope ps(n, RH_PHASE_EVAL);
    RH_HIP(rh::launch_eval(d, x, u, lam, y, true, st));
    RH_HIP(rh::launch_assemble_k(d, sig_x, sig_u, sig_s, st));
    if (r) RH_HIP(rh::launch_rtilde(d, r, sig_s, st));
  }
  {
    PhaseScope ps(n, RH_PHASE_REFACTOR);
    RH_HIP(rh::launch_refactor(d, st));
  }
  const int ncols = d.nu + (r ? 1 : 0);
  {
    PhaseScope ps(n, RH_PHASE_CONDENSE);
    RH_HIP(rh::launch_condense(d, 0, ncols, n->width, n->lds, r, K, long(ldk), rhs, st));
  }
  {
    PhaseScope ps(n, RH_PHASE_SYMMETRIZE);
    RH_HIP(rh::launch_symmetrize(K, long(ldk), d.nu, st));
  }
  n->condensed = true;
  n->rhs_cols = r != nullptr;
  return RH_OK;
}

rh_status rh_solve_condensed_kkt(rh_net* n, double* K, int64_t ldk, double delta_w,
                                 const double* rhs, const double* r, double* p,
                                 int32_t* dev_status) {
  if (!n || !K || !rhs || !r || !p) return RH_ERR_ARG;
  if (ldk < n->s.nu || !(delta_w >= 0.0)) return RH_ERR_ARG;
  if (!n->condensed) return RH_ERR_STATE;
  const auto& d = n->d;
  // the backward substitution keeps the right-hand side in LDS
  if (size_t((d.nu + 31) / 32) * 32 * sizeof(double) + 25 * 1024 > size_t(rh::max_lds_bytes()))
    return RH_ERR_ARG;
  hipStream_t st = n->stream;
  RH_HIP(hipMemcpyAsync(n->bwork, rhs, sizeof(double) * d.nu, hipMemcpyDeviceToDevice, st));
  {
    // L y = b is solved into p[0:nu], then L^T p_u = y in place
    PhaseScope ps(n, RH_PHASE_CHOLESKY);
    RH_HIP(rh::launch_cholesky_solve(K, long(ldk), d.nu, delta_w, n->bwork, p, n->cinv, n->lrow,
                                     n->status, st));
  }
  {
    PhaseScope ps(n, RH_PHASE_RECOVER);
    if (n->rhs_cols) {
      // p_x = Z p_u + d, p_lambda = -(Psi p_u + Psi_rhs) from the columns the
      // condensation stored (same r as the condensation's right-hand side)
      RH_HIP(rh::launch_recover_stored(d, p, st));
    } else {
      RH_HIP(rh::launch_rtilde(d, r, n->sig_s, st));
      RH_HIP(rh::launch_recover(d, p, r, p, st));
    }
    RH_HIP(rh::launch_finish_step(d, r, n->sig_s, p, st));
  }
  if (dev_status)
    RH_HIP(hipMemcpyAsync(dev_status, n->status, 2 * sizeof(int), hipMemcpyDeviceToDevice, st));
  int hs[4];
  RH_HIP(hipMemcpyAsync(hs, n->status, sizeof(hs), hipMemcpyDeviceToHost, st));
  RH_HIP(hipStreamSynchronize(st));
  if (hs[0] != 0) return RH_NOT_POSDEF;
  if (hs[2] != 0) return RH_SMALL_PIVOT;
  return RH_OK;
}

rh_status rh_profile_enable(rh_net* n, int32_t on) {
  if (!n) return RH_ERR_ARG;
  for (auto& t : n->timers) {
    drain(t);
    t.ms = 0.0;
    t.calls = 0;
  }
  n->profiling = on != 0;
  n->d.trace = n->profiling ? n->trace : nullptr;
  return RH_OK;
}

rh_status rh_profile_kernel_trace(rh_net* n, int64_t* ticks) {
  if (!n || !ticks) return RH_ERR_ARG;
  RH_HIP(hipStreamSynchronize(n->stream));
  long long h[256];
  RH_HIP(hipMemcpy(h, n->trace, sizeof(h), hipMemcpyDeviceToHost));
  for (int k = 0; k < 256; ++k) ticks[k] = h[k];
  return RH_OK;
}

rh_status rh_profile_read(rh_net* n, double* ms, int64_t* calls) {
  if (!n) return RH_ERR_ARG;
  for (int k = 0; k < RH_NPHASES; ++k) {
    drain(n->timers[k]);
    if (ms) ms[k] = n->timers[k].ms;
    if (calls) calls[k] = n->timers[k].calls;
  }
  return RH_OK;
}

}  // extern "C"
