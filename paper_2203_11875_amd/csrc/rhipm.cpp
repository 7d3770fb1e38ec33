// C ABI of the condensation hot path (declarations and contracts in rhipm.h).
#include "rhipm.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <memory>
#include <new>
#include <type_traits>
#include <vector>

#include "analysis.hpp"
#include "device.hpp"
#include "ipm.hpp"
#include "redlin.hpp"

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
  double* pf_scal = nullptr;  // power-flow residual of the last check (pinned host memory)
  // second stream: K assembly and rt run beside the refactorisation (which
  // occupies one work-group); events fork and join it
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  bool condensed = false;
  bool rhs_cols = false;     // the last condensation stored the right-hand-side column
  double* sig_s = nullptr;   // copy of Sigma_s from the last condensation
  double* bwork = nullptr;   // Cholesky right-hand-side work copy
  double* cinv = nullptr;    // 32 x 32 diagonal blocks of the Cholesky factor: inverses, then factors
  double* lrow = nullptr;    // the Cholesky factor by row blocks (backward substitution)
  int* status = nullptr;
  int* hstatus = nullptr;    // pinned host copy of the status words (the solve's last kernel writes it)
  long long* trace = nullptr;
  size_t panel_cap = 0;
  // objective scale (rh_set_objective_scale): unscaled cost data
  double obj_scale = 1.0;
  std::vector<double> c2, c1, c0, k_cdiag;
  double c2_ref = 0.0, c1_ref = 0.0, cost_rank1 = 0.0;
  // variable and slack bounds in the natural order (+-inf where none), for
  // the interior-point driver
  std::vector<double> wl, wu, sl, su;
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
// Networks with at least this many states refactorise level by level over
// many work-groups when they take the staged refactorisation.
constexpr int kStagedPerLevelStates = 4096;

#define RH_HIP(expr)                              \
  do {                                            \
    if ((expr) != hipSuccess) return RH_ERR_HIP;  \
  } while (0)

}  // namespace

struct rh_batch {
  std::vector<rh_net*> nets;
  hipStream_t stream = nullptr;
  hipGraph_t graph = nullptr;          // captured condensation + solve (rh_batch_capture)
  hipGraphExec_t graph_exec = nullptr;
  rh::BatchShape shape;
  rh::DevNet* d_nets = nullptr;
  rh::BatchArg* d_args = nullptr;
  int2* d_tiles = nullptr;
  int* d_status = nullptr;   // 5 status words per instance (pinned host memory)
  std::vector<rh::DevNet> h_nets;
  std::vector<rh::BatchArg> h_args;
  std::vector<char> up_nets, up_args;   // bytes of the last upload of h_nets, h_args
  // lockstep interior-point solvers (rh_ipm_batch_step): their device
  // descriptors with the reductions redirected to batch-wide arrays, the
  // evaluation arguments at the iterates and at the trial points, and the
  // per-instance scalars
  std::vector<unsigned long long> ipm_solvers;   // ids of the bound solvers
  rh::IpmDev* d_ipm = nullptr;
  rh::BatchArg *d_eargs = nullptr, *d_targs = nullptr;
  double* d_sc = nullptr;
  double *d_red = nullptr, *d_f = nullptr;   // pinned host memory, written by the kernels
  std::vector<double> h_sc, h_red, h_f;
  int max_vec = 0;
};

namespace {

rh_status upload_sweep(rh_net* n, const rh::Sweep& s, rh::DevSweep& d) {
  d.nlev = s.nlev;
  RH_TRY(upload(n, s.lev_ptr, &d.lev_ptr));
  RH_TRY(upload(n, s.rows, &d.rows));
  d.nstep = s.ks_nstep;
  d.ngrp[0] = rh::wave_groups(s, rh::kCondWaves);
  d.ngrp[1] = rh::wave_groups(s, rh::kCondWavesWide);
  d.unit = s.has_diag ? 0 : 1;
  return RH_OK;
}

// Which sweeps run on all waves of a condensation work-group of kCondWaves
// waves (bit k: L, U, U^T, L^T). A group of same-level steps, one per wave
// and then a barrier, took about 1.6 times a single-wave step with one
// work-group per CU and about 2.3 times with several (the waves of two
// work-groups then share SIMDs), measured on the 9241- and 1354-bus networks;
// a sweep is spread over the waves where its groups, weighted so, are fewer
// than its steps.
int sweep_grouping(const rh::DevNet& d, int nwv, int ntile, size_t lds_max) {
  const size_t per_wg = rh::condense_lds_bytes(d, 1, true, nwv);
  const long by_lds = per_wg ? long(lds_max / per_wg) : 1;
  const long cus = rh::device_cus();
  const long per_cu = std::min(by_lds, (ntile + cus - 1) / cus);
  const double f = per_cu <= 1 ? 1.6 : 2.3;
  const rh::DevSweep* sws[4] = {&d.sl, &d.su, &d.sut, &d.slt};
  int mask = 0;
  for (int k = 0; k < 4; ++k)
    if (f * sws[k]->ngrp[rh::wave_index(nwv)] < double(sws[k]->nstep)) mask |= 1 << k;
  return mask;
}

// Condensation records for launch width W (see rh::CondenseRecords).
rh_status upload_condense_records(rh_net* n, int W) {
  rh::DevNet& d = n->d;
  rh::CondenseRecords R;
  rh::build_condense_records(n->s, W, R);
  if (R.steps.size() >= size_t(1) << 31 || R.kstr.size() >= size_t(1) << 31) return RH_ERR_ARG;
  const double* pd;
  RH_TRY(upload(n, R.steps, &pd));
  d.lblk = const_cast<double*>(pd);
  rh::DevSweep* dsw[4] = {&d.sl, &d.su, &d.sut, &d.slt};
  for (int k = 0; k < 4; ++k) {
    RH_TRY(upload(n, R.meta[k], &dsw[k]->meta));
    for (int c = 0; c < 2; ++c) {
      RH_TRY(upload(n, R.gmeta[c][k], &dsw[k]->gmeta[c]));
      if (dsw[k]->ngrp[c] != R.ngrp[c][k]) return RH_ERR_ARG;
    }
  }
  d.tr_n = int(R.tr_dst.size());
  d.trd_n = int(R.trd_dst.size());
  RH_TRY(upload(n, R.tr_dst, &d.tr_dst));
  RH_TRY(upload(n, R.tr_src, &d.tr_src));
  RH_TRY(upload(n, R.trd_dst, &d.trd_dst));
  RH_TRY(upload(n, R.trd_src, &d.trd_src));
  RH_TRY(upload(n, R.kstr, &pd));
  d.kstr = const_cast<double*>(pd);
  RH_TRY(upload(n, R.gstr, &pd));
  d.gstr = const_cast<double*>(pd);
  RH_TRY(upload(n, R.kdst, &d.kdst));
  RH_TRY(upload(n, R.krt_dst, &d.krt_dst));
  RH_TRY(upload(n, R.gdst, &d.gdst));
  RH_TRY(upload(n, R.hpos, &d.hpos));
  RH_TRY(upload(n, R.grow, &d.grow));
  RH_TRY(upload(n, R.lsk_ptr, &d.lsk_ptr));
  RH_TRY(upload(n, R.lsk_meta, &d.lsk_meta));
  for (int c = 0; c < 2; ++c) {
    RH_TRY(upload(n, R.lsk_gptr[c], &d.lsk_gptr[c]));
    RH_TRY(upload(n, R.lsk_gmeta[c], &d.lsk_gmeta[c]));
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
  info->steps_lower = s.sl.ks_nstep;
  info->sweep_steps = s.sl.ks_nstep + s.su.ks_nstep + s.sut.ks_nstep + s.slt.ks_nstep;
  info->refactor_ops = s.refactor_ops;
  info->max_lu_row = s.max_row;
  info->max_row_ops = s.max_row_ops;
  info->refactor_kernel = s.rw_ok ? 0 : 1;
  info->refactor_split = s.rw_ok ? s.rw_split : 0;
  info->steps_l = s.sl.ks_nstep;
  info->steps_u = s.su.ks_nstep;
  info->steps_ut = s.sut.ks_nstep;
  info->steps_lt = s.slt.ks_nstep;
  info->groups_l = rh::wave_groups(s.sl, rh::kCondWaves);
  info->groups_u = rh::wave_groups(s.su, rh::kCondWaves);
  info->groups_ut = rh::wave_groups(s.sut, rh::kCondWaves);
  info->groups_lt = rh::wave_groups(s.slt, rh::kCondWaves);
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
  n->c2.assign(desc.c2, desc.c2 + s.ng);
  n->c1.assign(desc.c1, desc.c1 + s.ng);
  n->c0.assign(desc.c0, desc.c0 + s.ng);
  n->k_cdiag = s.k_cdiag;
  n->c2_ref = d.c2_ref;
  n->c1_ref = d.c1_ref;
  n->cost_rank1 = d.cost_rank1;
  {
    // bounds: theta free, Vm in [vmin, vmax], Pg in [pmin, pmax]; h = (Pg_ref,
    // Qg, |S_from|^2, |S_to|^2) in [(pmin_ref, qmin, -inf, -inf), (pmax_ref,
    // qmax, rate^2, rate^2)] and s = -h
    const double inf = HUGE_VAL;
    n->wl.assign(s.nw, -inf);
    n->wu.assign(s.nw, inf);
    for (int k = 0; k < s.nu; ++k) {
      const int r = s.u_ref[k];
      n->wl[k] = s.u_kind[k] == 1 ? desc.vmin[r] : desc.pmin[r];
      n->wu[k] = s.u_kind[k] == 1 ? desc.vmax[r] : desc.pmax[r];
    }
    for (int k = 0; k < s.nx; ++k)
      if (s.x_kind[k] == 1) {
        n->wl[s.nu + k] = desc.vmin[s.x_bus[k]];
        n->wu[s.nu + k] = desc.vmax[s.x_bus[k]];
      }
    std::vector<double> hl(s.m, -inf), hu(s.m, inf);
    hl[0] = desc.pmin[s.ref_gen];
    hu[0] = desc.pmax[s.ref_gen];
    for (int g = 0; g < s.ng; ++g) {
      hl[1 + g] = desc.qmin[g];
      hu[1 + g] = desc.qmax[g];
    }
    for (int l = 0; l < s.nl; ++l) {
      const int kl = s.lim_of_line[l];
      if (kl < 0) continue;
      hu[1 + s.ng + kl] = desc.rate[l] * desc.rate[l];
      hu[1 + s.ng + s.nlim + kl] = desc.rate[l] * desc.rate[l];
    }
    n->sl.resize(s.m);
    n->su.resize(s.m);
    for (int j = 0; j < s.m; ++j) {
      n->sl[j] = -hu[j];
      n->su[j] = -hl[j];
    }
  }
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
  RH_TRY(upload(n, s.kst.end, &d.kb_end));
  d.kst_nbat = s.kst.nbat;
  d.kb_n = int(s.kst.end.size());
  RH_TRY(upload(n, s.gst.end, &d.gt_end));
  d.gst_nbat = s.gst.nbat;
  d.gt_nb = int(s.gst.end.size());
  d.rw_ok = s.rw_ok ? 1 : 0;
  d.rw_nnz_u = s.rw_nnz_u;
  d.rw_nlev = s.sl.nlev;
  d.rw_wbeg = d.rw_levend = d.rw_rec = d.rw_lane = d.rw_ustart = d.rw_lanelu = nullptr;
  d.rw_ntask = 0;
  d.rw_lane_pad = 0;
  d.rw_split = s.rw_ok ? s.rw_split : 0;
  d.rw_split_grid = s.rw_split_grid;
  // the staged refactorisation of a large network runs one launch per level,
  // each level's rows spread over as many work-groups as its row groups need
  d.rf_per_level = (!s.rw_ok && s.nx >= kStagedPerLevelStates) ? 1 : 0;
  d.rf_level_grid = 1;
  for (int l = 0; l < s.sl.nlev; ++l) {
    const int rows = s.sl.lev_ptr[l + 1] - s.sl.lev_ptr[l];
    const int groups = 1024 / s.rf_lmeta[6 * l];
    d.rf_level_grid = std::max(d.rf_level_grid, (rows + groups - 1) / groups);
  }
  if (s.rw_ok) {
    d.rw_ntask = int(s.rw_rec.size()) / rh::kRwRec - 1;
    d.rw_lane_pad = int(s.rw_lane.size()) - 64;
    RH_TRY(upload(n, s.rw_wbeg, &d.rw_wbeg));
    RH_TRY(upload(n, s.rw_levend, &d.rw_levend));
    RH_TRY(upload(n, s.rw_rec, &d.rw_rec));
    RH_TRY(upload(n, s.rw_lane, &d.rw_lane));
    RH_TRY(upload(n, s.rw_ustart, &d.rw_ustart));
    RH_TRY(upload(n, s.rw_lanelu, &d.rw_lanelu));
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
  RH_TRY(alloc(n, rh::chol_inv_doubles(s.nu), &n->cinv));
  RH_TRY(alloc(n, rh::chol_lrow_doubles(s.nu), &n->lrow));
  RH_TRY(alloc(n, 8, &n->status));
  RH_HIP(hipHostMalloc(reinterpret_cast<void**>(&n->hstatus), 8 * sizeof(int), hipHostMallocCoherent));
  RH_TRY(alloc(n, 512, &n->trace));
  RH_HIP(hipMemset(n->trace, 0, 512 * sizeof(long long)));
  d.trace = nullptr;
  d.status = n->status;
  RH_HIP(hipMemset(n->status, 0, 8 * sizeof(int)));
  // launch shape of the condensation
  const size_t lds_max = size_t(rh::max_lds_bytes());
  int want = opts && opts->panel_width > 0 ? opts->panel_width : 1;
  if (want != 1 && want != 2 && want != 3 && want != 4 && want != 8) return RH_ERR_ARG;
  bool lds = !opts || opts->lds_panel != 0;
  if (opts && (opts->lds_panel < 0 || opts->lds_panel > 2)) return RH_ERR_ARG;
  // lds_panel 2: the sweep metadata read from global memory (one column per
  // work-group) even where it would fit beside the panel
  if (opts && opts->lds_panel == 2) {
    if (want != 1) return RH_ERR_ARG;
    d.meta_global = 1;
    if (rh::condense_lds_bytes(d, 1, true, 1) > lds_max) {
      d.meta_global = 0;
      lds = false;
    }
  }
  const int want_nw = opts ? opts->cond_waves : 0;
  if (want_nw != 0 && want_nw != 1 && want_nw != rh::kCondWavesPair && want_nw != rh::kCondWaves &&
      want_nw != rh::kCondWavesWide)
    return RH_ERR_ARG;
  const int want_grp = opts ? opts->sweep_grouping : 0;
  if (want_grp < 0 || want_grp > 16) return RH_ERR_ARG;
  if (lds && rh::condense_lds_bytes(d, want, true, 1) > lds_max) {
    // keep the panels in LDS with a narrower tile if possible, then with the
    // sweep metadata left in global memory (one column per work-group)
    int w = want;
    while (w > 1 && rh::condense_lds_bytes(d, w, true, 1) > lds_max) w = (w == 8 ? 4 : w - 1);
    if (rh::condense_lds_bytes(d, w, true, 1) <= lds_max) {
      want = w;
    } else {
      d.meta_global = 1;
      if (rh::condense_lds_bytes(d, 1, true, 1) <= lds_max) {
        want = 1;
      } else {
        d.meta_global = 0;
        lds = false;
      }
    }
  }
  // waves per work-group: several only for one column with its panel in LDS;
  // the record streams split over the waves, each sweep runs on all of them
  // or on one (sweep_grouping; always one with two waves). By default eight
  // where the panel fills the LDS (one work-group per CU; the 9241-bus
  // condensation call took 6.1 ms with one wave, 3.8 ms with four, 3.3 ms
  // with eight), else two (two or three work-groups per CU: the kernel took
  // 111 us with one wave, 104 us with two and 139 us with four at 1354
  // buses, where the sweeps on one wave of a four-wave work-group ran
  // slower than alone)
  d.cond_nw = 1;
  d.sweep_grouped = 0;
  if (lds && want == 1) {
    const int pick = want_nw != 0 ? want_nw : (d.meta_global ? rh::kCondWavesWide : rh::kCondWavesPair);
    if (pick > 1 && rh::condense_lds_bytes(d, 1, true, pick) <= lds_max) {
      d.cond_nw = pick;
      d.sweep_grouped = pick == rh::kCondWavesPair ? 0
                        : want_grp                 ? want_grp - 1
                                                   : sweep_grouping(d, pick, s.nu + 1, lds_max);
      if (rh::condense_lds_bytes(d, 1, true, pick) > lds_max) d.sweep_grouped = 0;
    }
  }
  n->width = want;
  n->lds = lds;
  RH_TRY(upload_condense_records(n, want));
  rh::prepare_lds_kernels();
  d.panel = nullptr;
  d.panel_doubles = 0;
  const size_t ntile = (size_t(s.nu) + 1 + want - 1) / want;
  if (!lds) {
    d.panel_doubles = ntile * (size_t(s.nw) + 1) * want;
    RH_TRY(alloc(n, d.panel_doubles, &d.panel));
  }
  RH_TRY(alloc(n, ntile * size_t(s.nw) * want, &d.hscr));
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

rh_status rh_symbolic_check_condense(const rh_symbolic* sym, int32_t width, uint64_t seed,
                                     double* max_rel_err) {
  if (!sym || !max_rel_err || (width != 1 && width != 2 && width != 3 && width != 4 && width != 8))
    return RH_ERR_ARG;
  return rh::host_check_condense(sym->s, width, seed, 3, max_rel_err);
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
  if (st == RH_OK &&
      (hipStreamCreateWithFlags(&n->side, hipStreamNonBlocking) != hipSuccess ||
       hipEventCreateWithFlags(&n->ev_fork, hipEventDisableTiming) != hipSuccess ||
       hipEventCreateWithFlags(&n->ev_join, hipEventDisableTiming) != hipSuccess))
    st = RH_ERR_HIP;
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
  if (n->side) (void)hipStreamSynchronize(n->side);
  for (auto& t : n->timers)
    for (auto& e : t.ev) (void)hipEventDestroy(e);
  if (n->ev_fork) (void)hipEventDestroy(n->ev_fork);
  if (n->ev_join) (void)hipEventDestroy(n->ev_join);
  if (n->side) (void)hipStreamDestroy(n->side);
  for (void* p : n->allocs) (void)hipFree(p);
  if (n->hstatus) (void)hipHostFree(n->hstatus);
  if (n->pf_scal) (void)hipHostFree(n->pf_scal);
  delete n;
}

rh_status rh_get_info(const rh_net* n, rh_info* info) {
  if (!n || !info) return RH_ERR_ARG;
  fill_info(n->s, info);
  info->panel_width = n->width;
  info->lds_panel = n->lds ? (n->d.meta_global ? 2 : 1) : 0;
  info->cond_waves = n->d.cond_nw;
  info->sweep_grouped = n->d.sweep_grouped;
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

rh_status rh_batch_create(rh_net* const* nets, int32_t count, void* hip_stream,
                          rh_batch** out) {
  if (!nets || count < 1 || !out) return RH_ERR_ARG;
  *out = nullptr;
  auto* b = new rh_batch();
  b->stream = static_cast<hipStream_t>(hip_stream);
  rh::BatchShape& sh = b->shape;
  sh.count = count;
  std::vector<int2> tiles;
  const size_t lds_max = size_t(rh::max_lds_bytes());
  std::vector<int> cls_of(count, -1);   // condensation class of each member
  for (int i = 0; i < count; ++i) {
    rh_net* n = nets[i];
    if (!n) { delete b; return RH_ERR_ARG; }
    for (size_t c = 0; c < sh.cls.size(); ++c)
      if (sh.cls[c].width == n->width && sh.cls[c].lds == n->lds) cls_of[i] = int(c);
    if (cls_of[i] < 0) {
      rh::CondClass c;
      c.width = n->width;
      c.lds = n->lds;
      sh.cls.push_back(c);
      cls_of[i] = int(sh.cls.size()) - 1;
    }
    const rh::DevNet& d = n->d;
    b->nets.push_back(n);
    sh.max_lines = std::max(sh.max_lines, std::max(d.nl, d.nu));
    sh.max_dst = std::max(sh.max_dst, d.d_total);
    sh.max_nnz_k = std::max(sh.max_nnz_k, d.nnz_k);
    sh.max_nw = std::max(sh.max_nw, d.nw);
    sh.max_nx = std::max(sh.max_nx, d.nx);
    sh.max_nu = std::max(sh.max_nu, d.nu);
    sh.max_m = std::max(sh.max_m, d.m);
    if (d.rw_ok) {
      sh.any_wave = true;
      sh.max_split = std::max(sh.max_split, d.rw_split);
      sh.max_split_grid = std::max(sh.max_split_grid, d.rw_split_grid);
      sh.lds_wave = std::max(sh.lds_wave, size_t(d.rw_nnz_u + 1 + d.nx) * sizeof(double) +
                                              size_t(rh::kRwWaves) * d.rw_nlev * sizeof(int));
    } else {
      if (d.rf_per_level) {
        sh.max_staged_levels = std::max(sh.max_staged_levels, d.rf_nlev);
        sh.max_staged_grid = std::max(sh.max_staged_grid, d.rf_level_grid);
      } else {
        sh.any_staged = true;
      }
      sh.lds_staged = std::max(sh.lds_staged, size_t(d.rf_lds_doubles) * sizeof(double));
    }
    sh.orders.push_back(d.nu);
  }
  // one condensation launch per class, its members' tiles contiguous. Within
  // a class one panel mode: the sweep metadata of every member is read from
  // global memory when one member's panel fills the LDS; several waves per
  // work-group then, or when every member of the class runs several (their
  // common count)
  bool lds_ok = sh.lds_wave <= lds_max && sh.lds_staged <= lds_max;
  for (size_t ci = 0; ci < sh.cls.size(); ++ci) {
    rh::CondClass& c = sh.cls[ci];
    c.tile0 = int(tiles.size());
    int common_nw = -1;
    // every member's last tile (the right-hand-side column's, the longest:
    // full L sweep, dense fill) first, then the others
    for (int i = 0; i < count; ++i)
      if (cls_of[i] == int(ci))
        tiles.push_back(int2{i, (nets[i]->d.nu + 1 + c.width - 1) / c.width - 1});
    for (int i = 0; i < count; ++i) {
      if (cls_of[i] != int(ci)) continue;
      const rh::DevNet& d = nets[i]->d;
      c.meta_global = c.meta_global || (c.lds && d.meta_global != 0);
      common_nw = common_nw < 0 || common_nw == d.cond_nw ? d.cond_nw : 0;
      const int ntile = (d.nu + 1 + c.width - 1) / c.width;
      for (int t = 0; t + 1 < ntile; ++t) tiles.push_back(int2{i, t});
    }
    c.ntiles = int(tiles.size()) - c.tile0;
    const bool all_nw = c.lds && c.width == 1 && common_nw > 1;
    auto lds_for = [&](int nw) {
      size_t m = 0;
      for (int i = 0; i < count; ++i) {
        if (cls_of[i] != int(ci)) continue;
        rh::DevNet dd = nets[i]->d;
        dd.meta_global = c.meta_global ? 1 : 0;
        m = std::max(m, rh::condense_lds_bytes(dd, c.width, c.lds, nw));
      }
      return m;
    };
    c.nw = 1;
    const int want_b = all_nw ? common_nw : rh::kCondWavesWide;
    if (c.lds && c.width == 1 && (c.meta_global || all_nw) && lds_for(want_b) <= lds_max)
      c.nw = want_b;
    c.lds_bytes = lds_for(c.nw);
    lds_ok = lds_ok && c.lds_bytes <= lds_max;
  }
  if (!lds_ok) {
    delete b;
    return RH_ERR_ARG;
  }
  b->h_nets.resize(count);
  b->h_args.resize(count);
  if (hipMalloc(&b->d_nets, sizeof(rh::DevNet) * count) != hipSuccess ||
      hipMalloc(&b->d_args, sizeof(rh::BatchArg) * count) != hipSuccess ||
      hipMalloc(&b->d_tiles, sizeof(int2) * tiles.size()) != hipSuccess ||
      hipHostMalloc(reinterpret_cast<void**>(&b->d_status), sizeof(int) * 5 * count,
                    hipHostMallocCoherent) != hipSuccess) {
    rh_batch_destroy(b);
    return RH_ERR_OOM;
  }
  if (hipMemcpy(b->d_tiles, tiles.data(), sizeof(int2) * tiles.size(), hipMemcpyHostToDevice) !=
      hipSuccess) {
    rh_batch_destroy(b);
    return RH_ERR_HIP;
  }
  *out = b;
  return RH_OK;
}

void rh_batch_destroy(rh_batch* b) {
  if (!b) return;
  if (b->stream) (void)hipStreamSynchronize(b->stream);
  else (void)hipDeviceSynchronize();
  if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  (void)hipFree(b->d_nets);
  (void)hipFree(b->d_args);
  (void)hipFree(b->d_tiles);
  if (b->d_status) (void)hipHostFree(b->d_status);
  for (void* q : {(void*)b->d_ipm, (void*)b->d_eargs, (void*)b->d_targs, (void*)b->d_sc})
    if (q) (void)hipFree(q);
  for (void* q : {(void*)b->d_red, (void*)b->d_f})   // pinned host memory
    if (q) (void)hipHostFree(q);
  delete b;
}

namespace {
// the instances' own streams may still run earlier work on their buffers
rh_status batch_wait_instances(rh_batch* b) {
  std::vector<hipStream_t> seen;
  for (rh_net* n : b->nets)
    if (n->stream != b->stream && std::find(seen.begin(), seen.end(), n->stream) == seen.end()) {
      seen.push_back(n->stream);
      RH_HIP(hipStreamSynchronize(n->stream));
    }
  return RH_OK;
}

// the instances' current device descriptors (profiling or new loads change
// them between calls) and the per-call arguments, to the device
rh_status batch_upload(rh_batch* b) {
  for (size_t i = 0; i < b->nets.size(); ++i) {
    rh_net* n = b->nets[i];
    b->h_nets[i] = n->d;
    rh::BatchArg& a = b->h_args[i];
    a.sig_s_keep = n->sig_s;
    a.bwork = n->bwork;
    a.cinv = n->cinv;
    a.lrow = n->lrow;
    a.status = n->status;
    a.nu = n->d.nu;
    a.m = n->d.m;
  }
  // the kernels only read these arrays: bytes equal to the last upload are
  // already on the device (a replay with the same arguments copies nothing)
  const size_t nb = sizeof(rh::DevNet) * b->nets.size(), ab = sizeof(rh::BatchArg) * b->nets.size();
  if (b->up_nets.size() != nb || std::memcmp(b->up_nets.data(), b->h_nets.data(), nb) != 0) {
    RH_HIP(hipMemcpyAsync(b->d_nets, b->h_nets.data(), nb, hipMemcpyHostToDevice, b->stream));
    b->up_nets.assign(reinterpret_cast<const char*>(b->h_nets.data()),
                      reinterpret_cast<const char*>(b->h_nets.data()) + nb);
  }
  if (b->up_args.size() != ab || std::memcmp(b->up_args.data(), b->h_args.data(), ab) != 0) {
    RH_HIP(hipMemcpyAsync(b->d_args, b->h_args.data(), ab, hipMemcpyHostToDevice, b->stream));
    b->up_args.assign(reinterpret_cast<const char*>(b->h_args.data()),
                      reinterpret_cast<const char*>(b->h_args.data()) + ab);
  }
  return RH_OK;
}
}  // namespace

rh_status rh_batch_condense(rh_batch* b, const rh_batch_condense_item* items) {
  if (!b || !items) return RH_ERR_ARG;
  for (size_t i = 0; i < b->nets.size(); ++i) {
    const rh_batch_condense_item& it = items[i];
    if (!it.x || !it.u || !it.lam || !it.y || !it.sig_x || !it.sig_u || !it.sig_s || !it.r ||
        !it.K || !it.rhs || it.ldk < b->nets[i]->d.nu)
      return RH_ERR_ARG;
    rh::BatchArg& a = b->h_args[i];
    a = rh::BatchArg{};
    a.x = it.x; a.u = it.u; a.lam = it.lam; a.y = it.y;
    a.sig_x = it.sig_x; a.sig_u = it.sig_u; a.sig_s = it.sig_s; a.r = it.r;
    a.K = it.K; a.ldk = long(it.ldk); a.rhs = it.rhs;
  }
  RH_TRY(batch_wait_instances(b));
  RH_TRY(batch_upload(b));
  RH_HIP(rh::launch_batch_condense(b->d_nets, b->d_args, b->d_tiles, b->shape, b->stream));
  for (rh_net* n : b->nets) {
    n->condensed = true;
    n->rhs_cols = true;
  }
  return RH_OK;
}

namespace {
rh_status batch_statuses(rh_batch* b, int32_t* status);
}  // namespace

rh_status rh_batch_solve(rh_batch* b, const rh_batch_solve_item* items, int32_t* status) {
  if (!b || !items) return RH_ERR_ARG;
  for (size_t i = 0; i < b->nets.size(); ++i) {
    const rh_batch_solve_item& it = items[i];
    rh_net* n = b->nets[i];
    if (!it.K || !it.rhs || !it.r || !it.p || it.ldk < n->d.nu || !(it.delta_w >= 0.0))
      return RH_ERR_ARG;
    if (!n->condensed || !n->rhs_cols) return RH_ERR_STATE;
    rh::BatchArg& a = b->h_args[i];
    a = rh::BatchArg{};
    a.K = it.K; a.ldk = long(it.ldk); a.delta = it.delta_w; a.rhs = const_cast<double*>(it.rhs);
    a.r = it.r; a.p = it.p;
  }
  RH_TRY(batch_wait_instances(b));
  RH_TRY(batch_upload(b));
  RH_HIP(rh::launch_batch_solve(b->d_nets, b->d_args, b->shape, b->stream));
  return batch_statuses(b, status);
}

namespace {
rh_status batch_statuses(rh_batch* b, int32_t* status) {
  RH_HIP(rh::launch_batch_status(b->d_nets, int(b->nets.size()), b->d_status, b->stream));
  RH_HIP(hipStreamSynchronize(b->stream));
  const int* hs = b->d_status;   // pinned host memory, written by the status kernel
  rh_status worst = RH_OK;
  for (size_t i = 0; i < b->nets.size(); ++i) {
    rh_status si = RH_OK;
    if (hs[5 * i + 4] != 0) si = RH_ERR_STATE;
    else if (hs[5 * i + 2] != 0) si = RH_SMALL_PIVOT;
    else if (hs[5 * i] != 0) si = RH_NOT_POSDEF;
    if (status) status[i] = si;
    if (si != RH_OK && worst == RH_OK) worst = si;
  }
  return worst;
}

// condensation + solve arguments in one BatchArg per instance
rh_status batch_fill_step(rh_batch* b, const rh_batch_condense_item* ci,
                          const rh_batch_solve_item* si) {
  for (size_t i = 0; i < b->nets.size(); ++i) {
    const rh_batch_condense_item& c = ci[i];
    const rh_batch_solve_item& q = si[i];
    const int nu = b->nets[i]->d.nu;
    if (!c.x || !c.u || !c.lam || !c.y || !c.sig_x || !c.sig_u || !c.sig_s || !c.r || !c.K ||
        !c.rhs || c.ldk < nu || q.K != c.K || q.ldk != c.ldk || q.rhs != c.rhs || q.r != c.r ||
        !q.p || !(q.delta_w >= 0.0))
      return RH_ERR_ARG;
    rh::BatchArg& a = b->h_args[i];
    a = rh::BatchArg{};
    a.x = c.x; a.u = c.u; a.lam = c.lam; a.y = c.y;
    a.sig_x = c.sig_x; a.sig_u = c.sig_u; a.sig_s = c.sig_s; a.r = c.r;
    a.K = c.K; a.ldk = long(c.ldk); a.rhs = c.rhs; a.p = q.p; a.delta = q.delta_w;
  }
  return RH_OK;
}
}  // namespace

rh_status rh_batch_capture(rh_batch* b, const rh_batch_condense_item* citems,
                           const rh_batch_solve_item* sitems) {
  if (!b || !citems || !sitems || !b->stream) return RH_ERR_ARG;
  RH_TRY(batch_fill_step(b, citems, sitems));
  RH_TRY(batch_wait_instances(b));
  RH_TRY(batch_upload(b));
  RH_HIP(hipStreamSynchronize(b->stream));
  if (b->graph_exec) { (void)hipGraphExecDestroy(b->graph_exec); b->graph_exec = nullptr; }
  if (b->graph) { (void)hipGraphDestroy(b->graph); b->graph = nullptr; }
  RH_HIP(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
  hipError_t e1 = rh::launch_batch_condense(b->d_nets, b->d_args, b->d_tiles, b->shape, b->stream);
  hipError_t e2 = rh::launch_batch_solve(b->d_nets, b->d_args, b->shape, b->stream);
  hipGraph_t g = nullptr;
  hipError_t e3 = hipStreamEndCapture(b->stream, &g);
  if (e1 != hipSuccess || e2 != hipSuccess || e3 != hipSuccess || !g) {
    if (g) (void)hipGraphDestroy(g);
    return RH_ERR_HIP;
  }
  b->graph = g;
  if (hipGraphInstantiate(&b->graph_exec, g, nullptr, nullptr, 0) != hipSuccess) {
    b->graph_exec = nullptr;
    return RH_ERR_HIP;
  }
  return RH_OK;
}

rh_status rh_batch_replay(rh_batch* b, const rh_batch_condense_item* citems,
                          const rh_batch_solve_item* sitems, int32_t* status) {
  if (!b || !b->graph_exec) return RH_ERR_STATE;
  if (citems || sitems) {
    if (!citems || !sitems) return RH_ERR_ARG;
    RH_TRY(batch_fill_step(b, citems, sitems));
  }
  // refresh the device descriptors and arguments the graph's kernels read
  RH_TRY(batch_wait_instances(b));
  RH_TRY(batch_upload(b));
  RH_HIP(hipGraphLaunch(b->graph_exec, b->stream));
  for (rh_net* n : b->nets) {
    n->condensed = true;
    n->rhs_cols = true;
  }
  return batch_statuses(b, status);
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

}  // extern "C"

namespace {

// Condensation once the derivative values at (x, u, lambda, y) are in place
// (rh_condense_reduced_hessian after its evaluation; the interior-point
// driver after its own).
// Kcopy (optional, leading dimension ldk): receives the symmetrised K_cond
// as well (an interior-point solver's copy for inertia-correction retries).
rh_status condense_evaluated(rh_net* n, const double* sig_x, const double* sig_u,
                             const double* sig_s, const double* r, double* K, int64_t ldk,
                             double* rhs, double* Kcopy = nullptr) {
  const auto& d = n->d;
  hipStream_t st = n->stream;
  n->condensed = false;
  // K assembly (which also keeps a copy of Sigma_s for the recovery) and rt
  // on the side stream, beside the refactorisation; the condensation and
  // everything after it wait for both
  RH_HIP(hipEventRecord(n->ev_fork, st));
  RH_HIP(hipStreamWaitEvent(n->side, n->ev_fork, 0));
  RH_HIP(rh::launch_assemble_k(d, sig_x, sig_u, sig_s, n->sig_s, n->side));
  RH_HIP(rh::launch_rtilde(d, r, sig_s, n->side));   // r == NULL: rt = 0
  RH_HIP(hipEventRecord(n->ev_join, n->side));
  {
    PhaseScope ps(n, RH_PHASE_REFACTOR);
    RH_HIP(rh::launch_refactor(d, st));
  }
  RH_HIP(hipStreamWaitEvent(st, n->ev_join, 0));
  const int ncols = d.nu + (r ? 1 : 0);
  {
    PhaseScope ps(n, RH_PHASE_CONDENSE);
    RH_HIP(rh::launch_condense(d, 0, ncols, n->width, n->lds, r, K, long(ldk), rhs, st));
  }
  {
    PhaseScope ps(n, RH_PHASE_SYMMETRIZE);
    RH_HIP(rh::launch_symmetrize(K, long(ldk), d.nu, Kcopy, st));
  }
  n->condensed = true;
  n->rhs_cols = r != nullptr;
  return RH_OK;
}

}  // namespace

extern "C" {

rh_status rh_condense_reduced_hessian(rh_net* n, const double* x, const double* u,
                                      const double* lam, const double* y,
                                      const double* sig_x, const double* sig_u,
                                      const double* sig_s, const double* r,
                                      double* K, int64_t ldk, double* rhs) {
  if (!n || !x || !u || !lam || !y || !sig_x || !sig_u || !sig_s || !K) return RH_ERR_ARG;
  if (ldk < n->s.nu || (r && !rhs) || (rhs && !r)) return RH_ERR_ARG;
  {
    PhaseScope ps(n, RH_PHASE_EVAL);
    RH_HIP(rh::launch_eval(n->d, x, u, lam, y, true, n->stream));
  }
  return condense_evaluated(n, sig_x, sig_u, sig_s, r, K, ldk, rhs);
}

rh_status rh_set_objective_scale(rh_net* n, double scale) {
  if (!n || !(scale > 0.0) || !std::isfinite(scale)) return RH_ERR_ARG;
  auto& d = n->d;
  const size_t ng = n->c2.size();
  std::vector<double> c2(ng), c1(ng), c0(ng), kc(n->k_cdiag.size());
  for (size_t g = 0; g < ng; ++g) {
    c2[g] = scale * n->c2[g];
    c1[g] = scale * n->c1[g];
    c0[g] = scale * n->c0[g];
  }
  for (size_t k = 0; k < kc.size(); ++k) kc[k] = scale * n->k_cdiag[k];
  RH_HIP(hipStreamSynchronize(n->stream));
  RH_HIP(hipMemcpy(const_cast<double*>(d.c2), c2.data(), ng * sizeof(double), hipMemcpyHostToDevice));
  RH_HIP(hipMemcpy(const_cast<double*>(d.c1), c1.data(), ng * sizeof(double), hipMemcpyHostToDevice));
  RH_HIP(hipMemcpy(const_cast<double*>(d.c0), c0.data(), ng * sizeof(double), hipMemcpyHostToDevice));
  RH_HIP(hipMemcpy(const_cast<double*>(d.k_cdiag), kc.data(), kc.size() * sizeof(double),
                   hipMemcpyHostToDevice));
  d.c2_ref = scale * n->c2_ref;
  d.c1_ref = scale * n->c1_ref;
  d.cost_rank1 = scale * n->cost_rank1;
  n->obj_scale = scale;
  return RH_OK;
}

rh_status rh_solve_condensed_kkt(rh_net* n, double* K, int64_t ldk, double delta_w,
                                 const double* rhs, const double* r, double* p,
                                 int32_t* dev_status) {
  if (!n || !K || !rhs || !r || !p) return RH_ERR_ARG;
  if (ldk < n->s.nu || !(delta_w >= 0.0)) return RH_ERR_ARG;
  if (!n->condensed) return RH_ERR_STATE;
  const auto& d = n->d;
  hipStream_t st = n->stream;
  {
    // L y = rhs into the work copy (rhs itself is left as it is), then
    // L^T p_u = y into p[0:nu]
    PhaseScope ps(n, RH_PHASE_CHOLESKY);
    RH_HIP(rh::launch_cholesky_solve(K, long(ldk), d.nu, delta_w, rhs, n->bwork, p, n->cinv, n->lrow,
                                     n->status, st, n->profiling ? n->trace + 256 : nullptr));
  }
  {
    PhaseScope ps(n, RH_PHASE_RECOVER);
    if (n->rhs_cols) {
      // p_x = Z p_u + d, p_lambda = -(Psi p_u + Psi_rhs) from the columns the
      // condensation stored (same r as the condensation's right-hand side)
      RH_HIP(rh::launch_recover_stored(d, p, st));
    } else {
      RH_HIP(rh::launch_rtilde(d, r, n->sig_s, st));
      RH_HIP(rh::launch_recover(d, n->width, n->lds, p, r, p, st));
    }
    RH_HIP(rh::launch_finish_step(d, r, n->sig_s, p, n->hstatus, st));
  }
  if (dev_status)
    RH_HIP(hipMemcpyAsync(dev_status, n->status, 2 * sizeof(int), hipMemcpyDeviceToDevice, st));
  RH_HIP(hipStreamSynchronize(st));
  const int* hs = n->hstatus;   // written by the step's last kernel
  if (hs[4] != 0) return RH_ERR_STATE;   // condensation panels not at LDS address 0
  // a tiny static pivot makes G_x's factors, hence K_cond, unusable: it is
  // reported before the Cholesky's outcome
  if (hs[2] != 0) return RH_SMALL_PIVOT;
  if (hs[0] != 0) return RH_NOT_POSDEF;
  return RH_OK;
}

rh_status rh_cholesky_solve_noalloc(double* K, int64_t ldk, int32_t n, double delta_w,
                                    const double* b, double* x, int32_t* dev_status,
                                    void* hip_stream) {
  if (n < 0 || n > rh::kNoallocMaxOrder || !(delta_w >= 0.0) || !dev_status) return RH_ERR_ARG;
  if (n > 0 && (!K || !b || !x || ldk < n)) return RH_ERR_ARG;
  RH_HIP(rh::launch_cholesky_solve_noalloc(K, long(ldk), n, delta_w, b, x, dev_status,
                                           static_cast<hipStream_t>(hip_stream)));
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
  long long h[512];
  RH_HIP(hipMemcpy(h, n->trace, sizeof(h), hipMemcpyDeviceToHost));
  for (int k = 0; k < 512; ++k) ticks[k] = h[k];
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

// ---------------------------------------------------------------------------
// Interior-point driver (Algorithm 1, linearize-then-reduce). The host runs
// the scalar logic (barrier update, inertia correction, filter line search);
// every vector operation, evaluation, condensation and solve runs on the
// device and the host reads a few reduced scalars per stage.
// ---------------------------------------------------------------------------
namespace {

// Fixed constants of the method (the filter line search of Waechter and
// Biegler with a monotone barrier update; see rh_ipm_options).
constexpr double kKappaEps = 10.0, kKappaMu = 0.2, kThetaMu = 1.5, kTauMin = 0.99;
constexpr double kSMax = 100.0, kKappaSigma = 1e10, kBoundPush = 1e-2, kBoundFrac = 1e-2;
constexpr double kDelta0 = 1e-4, kDeltaMin = 1e-20, kDeltaMax = 1e40;
constexpr double kKwMinus = 1.0 / 3.0, kKwPlus = 8.0, kKwPlusBar = 100.0;
constexpr double kGammaTheta = 1e-5, kGammaPhi = 1e-8, kDeltaSw = 1.0, kSTheta = 1.1;
constexpr double kSPhi = 2.3, kEtaPhi = 1e-8, kGammaAlpha = 0.05;

}  // namespace

struct rh_ipm {
  rh_net* net = nullptr;
  unsigned long long id = 0;   // unique per solver created in this process
  rh_ipm_options opt{};
  rh::IpmDev v{};
  std::vector<void*> allocs;
  std::vector<void*> hallocs;   // pinned host memory (the reduction slots, objective values)
  double* K = nullptr;      // nu x nu condensed matrix (factored in place)
  double* Kc = nullptr;     // its copy for inertia-correction retries
  double* rhs = nullptr;
  double mu = 0.1, delta_last = 0.0, theta0 = -1.0, sigma_f = 1.0;
  std::vector<std::pair<double, double>> filt;
  long iter = 0;
  int nfin = 0;             // finite bounds of w and s
  bool converged = false;
};

namespace {

template <typename H, typename T>
rh_status ialloc(H* p, size_t count, T** out) {
  void* q = nullptr;
  if (hipMalloc(&q, std::max<size_t>(1, count) * sizeof(T)) != hipSuccess) return RH_ERR_OOM;
  p->allocs.push_back(q);
  *out = static_cast<T*>(q);
  return RH_OK;
}

// Pinned, coherent host memory for values that kernels write with plain
// stores and the host reads once the stream has drained (reduction slots,
// objective values): no copy back, no device-to-host transfer.
template <typename H, typename T>
rh_status halloc(H* p, size_t count, T** out) {
  void* q = nullptr;
  if (hipHostMalloc(&q, std::max<size_t>(1, count) * sizeof(T), hipHostMallocCoherent) != hipSuccess)
    return RH_ERR_OOM;
  p->hallocs.push_back(q);
  *out = static_cast<T*>(q);
  return RH_OK;
}

template <typename H, typename T>
rh_status iupload(H* p, const std::vector<T>& h, const T** out) {
  T* q = nullptr;
  RH_TRY(ialloc(p, h.size(), &q));
  if (!h.empty() && hipMemcpy(q, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess)
    return RH_ERR_HIP;
  *out = q;
  return RH_OK;
}

template <typename H>
void free_ipm(H* p) {
  for (void* q : p->allocs) (void)hipFree(q);
  p->allocs.clear();
  for (void* q : p->hallocs) (void)hipHostFree(q);
  p->hallocs.clear();
}

// Device vectors of an interior-point handle on network n (natural order,
// w = [u; x]): bounds, the generator of each Pg control, G_x by internal
// columns (for G^T lambda), iterate, multipliers, residual, step, trial point
// and reduction slots. nfin: finite bounds of w and s.
template <typename H>
rh_status setup_ipm_dev(H* p, rh_net* n, rh::IpmDev& v, int* nfin) {
  const rh::Symbolic& s = n->s;
  v.nu = s.nu;
  v.nx = s.nx;
  v.m = s.m;
  const int nw = s.nw, m = s.m, nx = s.nx, nu = s.nu;
  *nfin = 0;
  RH_TRY(iupload(p, n->wl, &v.wl));
  RH_TRY(iupload(p, n->wu, &v.wu));
  RH_TRY(iupload(p, n->sl, &v.sl));
  RH_TRY(iupload(p, n->su, &v.su));
  for (const auto* b : {&n->wl, &n->wu, &n->sl, &n->su})
    for (double x : *b) *nfin += std::isfinite(x) ? 1 : 0;
  {
    std::vector<int> ug(nu, -1);
    for (int k = 0; k < nu; ++k)
      if (s.u_kind[k] == 2) ug[k] = s.u_ref[k];
    RH_TRY(iupload(p, ug, &v.u_gen));
    // G_x by internal columns (transposed products with lambda)
    std::vector<std::vector<std::pair<int, int>>> cols(nx);
    for (int r = 0; r < nx; ++r)
      for (int e = s.gx_ptr[r]; e < s.gx_ptr[r + 1]; ++e)
        cols[s.iperm[s.gx_col[e]]].push_back({s.iperm[r], s.gx_lu[e]});
    std::vector<int> cptr(nx + 1, 0), crow, cpos;
    for (int c = 0; c < nx; ++c) {
      for (auto& q : cols[c]) {
        crow.push_back(q.first);
        cpos.push_back(q.second);
      }
      cptr[c + 1] = int(crow.size());
    }
    RH_TRY(iupload(p, cptr, &v.gx_cptr));
    RH_TRY(iupload(p, crow, &v.gx_crow));
    RH_TRY(iupload(p, cpos, &v.gx_cpos));
  }
  const size_t np = size_t(nw) + 2 * size_t(m) + nx;
  RH_TRY(ialloc(p, nw, &v.w));
  RH_TRY(ialloc(p, m, &v.s));
  RH_TRY(ialloc(p, nx, &v.lam));
  RH_TRY(ialloc(p, m, &v.y));
  RH_TRY(ialloc(p, nw, &v.zl));
  RH_TRY(ialloc(p, nw, &v.zu));
  RH_TRY(ialloc(p, m, &v.zsl));
  RH_TRY(ialloc(p, m, &v.zsu));
  RH_TRY(ialloc(p, nw, &v.gf));
  RH_TRY(ialloc(p, nw, &v.gl));
  RH_TRY(ialloc(p, nw, &v.sig_w));
  RH_TRY(ialloc(p, m, &v.sig_s));
  RH_TRY(ialloc(p, np, &v.r));
  RH_TRY(ialloc(p, np, &v.p));
  RH_TRY(ialloc(p, nw, &v.pzl));
  RH_TRY(ialloc(p, nw, &v.pzu));
  RH_TRY(ialloc(p, m, &v.pzsl));
  RH_TRY(ialloc(p, m, &v.pzsu));
  RH_TRY(ialloc(p, nw, &v.wt));
  RH_TRY(ialloc(p, m, &v.st));
  RH_TRY(halloc(p, rh::IR_NSLOT, &v.red));
  RH_TRY(halloc(p, 2, &v.f));
  return RH_OK;
}

// Reads the reduction slots (and the two objective values; both in pinned
// host memory) after the stream has drained.
rh_status read_red(rh_ipm* p, double* red, double* f) {
  RH_HIP(hipStreamSynchronize(p->net->stream));
  std::memcpy(red, p->v.red, sizeof(double) * rh::IR_NSLOT);
  if (f) std::memcpy(f, p->v.f, sizeof(double) * 2);
  return RH_OK;
}

// Scaled optimality error E_mu from the reductions of launch_ipm_stats.
double opt_error(const rh_ipm* p, const double* red, double mu) {
  const auto& v = p->v;
  const double sd = std::max(kSMax, (red[rh::IR_LYSUM] + red[rh::IR_ZSUM]) /
                                        std::max(1, v.nx + v.m + p->nfin)) / kSMax;
  const double sc = std::max(kSMax, red[rh::IR_ZSUM] / std::max(1, p->nfin)) / kSMax;
  const double ed = std::max(red[rh::IR_DUAL_W], v.m ? red[rh::IR_DUAL_S] : 0.0) / sd;
  const double ep = std::max(red[rh::IR_PRIM_G], v.m ? red[rh::IR_PRIM_H] : 0.0);
  const double ec =
      p->nfin ? std::max(red[rh::IR_DZ_MAX] - mu, mu - red[rh::IR_DZ_MIN]) / sc : 0.0;
  return std::max(ed, std::max(ep, ec));
}

void fill_info(const rh_ipm* p, rh_ipm_info* info, double obj, double inf_pr, double err,
               double alpha, double alpha_z, double delta, long trials) {
  if (!info) return;
  std::memset(info, 0, sizeof(*info));
  info->iter = p->iter;
  info->obj = obj;
  info->inf_pr = inf_pr;
  info->err = err;
  info->mu = p->mu;
  info->alpha_pr = alpha;
  info->alpha_du = alpha_z;
  info->delta_w = delta;
  info->ls_trials = trials;
  info->converged = p->converged ? 1 : 0;
  info->obj_scale = p->sigma_f;
}

// One iteration of Algorithm 1 in stages, so that a batch of solvers can run
// them in lockstep (rh_ipm_batch_step) with the condensation and the solve
// batched; rh_ipm_step runs the same stages for one solver.
struct IpmStep {
  double red[rh::IR_NSLOT] = {}, f2[2] = {}, f0 = 0.0, e0 = 0.0, mu = 0.0, delta = 0.0;
  double a_pri = 1.0, a_dual = 1.0, dphi = 0.0, theta = 0.0, phi = 0.0;
  double theta_max = 0.0, theta_min = 0.0, a_min = 0.0, alpha = 1.0;
  double rt[rh::IR_NSLOT] = {}, ft[2] = {};
  long trials = 0;
  bool ftype = false;
  bool done = false;      // the iteration ended (converged, failed or max_iter)
  rh_status code = RH_OK;
};

// Evaluation at the current iterate (launches only).
rh_status ipm_eval_launch(rh_ipm* p) {
  rh_net* n = p->net;
  // another solver on the same network may have changed the objective scale
  if (n->obj_scale != p->sigma_f) RH_TRY(rh_set_objective_scale(n, p->sigma_f));
  const auto& d = n->d;
  auto& v = p->v;
  hipStream_t st = n->stream;
  PhaseScope ps(n, RH_PHASE_EVAL);
  RH_HIP(rh::launch_eval(d, v.w + v.nu, v.w, v.lam, v.y, true, st));
  RH_HIP(rh::launch_eval_objective(d, v.w, v.f, st));
  RH_HIP(rh::launch_ipm_lag_grad(d, v, st));
  RH_HIP(rh::launch_ipm_stats(d, v, v.w, v.s, 1, st));
  return RH_OK;
}

// Convergence test, iteration limit and barrier update from the reductions
// of the evaluation in s.red, s.f2.
void ipm_begin_logic(rh_ipm* p, IpmStep& s, rh_ipm_info* info) {
  const double* red = s.red;
  s.f0 = s.f2[0];
  s.e0 = opt_error(p, red, 0.0);
  const double inf_pr = std::max(red[rh::IR_PRIM_G], red[rh::IR_PRIM_H]);
  if (s.e0 <= p->opt.tol) {
    p->converged = true;
    fill_info(p, info, s.f0 / p->sigma_f, inf_pr, s.e0, 0.0, 0.0, 0.0, 0);
    s.done = true;
    s.code = RH_OK;
    return;
  }
  if (p->iter >= p->opt.max_iter) {
    fill_info(p, info, s.f0 / p->sigma_f, inf_pr, s.e0, 0.0, 0.0, 0.0, 0);
    s.done = true;
    s.code = RH_NOT_CONVERGED;
    return;
  }
  // barrier update (monotone)
  for (int k = 0; k < 10; ++k) {
    if (opt_error(p, red, p->mu) > kKappaEps * p->mu) break;
    const double nm = std::max(p->opt.tol / 10.0, std::min(kKappaMu * p->mu, std::pow(p->mu, kThetaMu)));
    if (nm == p->mu) break;
    p->mu = nm;
    p->filt.clear();
  }
  s.mu = p->mu;
}

// Reads the evaluation's reductions, then the above, then residuals and Sigma.
rh_status ipm_begin(rh_ipm* p, IpmStep& s, rh_ipm_info* info) {
  RH_TRY(read_red(p, s.red, s.f2));
  ipm_begin_logic(p, s, info);
  if (!s.done) RH_HIP(rh::launch_ipm_prep(p->net->d, p->v, s.mu, p->net->stream));
  return RH_OK;
}

rh_status ipm_condense_single(rh_ipm* p) {
  rh_net* n = p->net;
  auto& v = p->v;
  const int nu = v.nu;
  return condense_evaluated(n, v.sig_w + nu, v.sig_w, v.sig_s, v.r, p->K, nu, p->rhs, p->Kc);
}

rh_status ipm_first_solve(rh_ipm* p) {
  return rh_solve_condensed_kkt(p->net, p->K, p->v.nu, 0.0, p->rhs, p->v.r, p->v.p, nullptr);
}

// Inertia correction after the first solve (delta_w = 0) returned `code`:
// K_cond + delta_w I from the saved copy until the factorisation succeeds.
rh_status ipm_factor(rh_ipm* p, IpmStep& s, rh_ipm_info* info, rh_status code) {
  rh_net* n = p->net;
  auto& v = p->v;
  const int nu = v.nu;
  s.delta = 0.0;
  if (code == RH_SMALL_PIVOT) {
    // the static pivots of G_x no longer hold at this iterate: no step is
    // taken from these factors (the iterate is left unchanged)
    fill_info(p, info, s.f0 / p->sigma_f, std::max(s.red[rh::IR_PRIM_G], s.red[rh::IR_PRIM_H]),
              s.e0, 0.0, 0.0, 0.0, 0);
    s.done = true;
    s.code = RH_SMALL_PIVOT;
    return RH_OK;
  }
  if (code == RH_NOT_POSDEF) {
    double delta = p->delta_last == 0.0 ? kDelta0 : std::max(kDeltaMin, kKwMinus * p->delta_last);
    for (;;) {
      RH_HIP(hipMemcpyAsync(p->K, p->Kc, sizeof(double) * size_t(nu) * nu,
                            hipMemcpyDeviceToDevice, n->stream));
      code = rh_solve_condensed_kkt(n, p->K, nu, delta, p->rhs, v.r, v.p, nullptr);
      if (code != RH_NOT_POSDEF) break;
      delta *= p->delta_last == 0.0 ? kKwPlusBar : kKwPlus;
      if (delta > kDeltaMax) {
        fill_info(p, info, s.f0 / p->sigma_f,
                  std::max(s.red[rh::IR_PRIM_G], s.red[rh::IR_PRIM_H]), s.e0, 0.0, 0.0, delta, 0);
        s.done = true;
        s.code = RH_NOT_CONVERGED;
        return RH_OK;
      }
    }
    p->delta_last = delta;
    s.delta = delta;
  }
  if (code < 0) return code;
  return RH_OK;
}

// bound-multiplier steps and the largest steps to the boundary
rh_status ipm_dir_launch(rh_ipm* p, IpmStep& s) {
  const double tau = std::max(kTauMin, 1.0 - s.mu);
  RH_HIP(rh::launch_ipm_dir(p->v, s.mu, tau, p->net->stream));
  return RH_OK;
}

// line-search constants of the filter method from the reductions rd of
// launch_ipm_dir
void ipm_dir_logic(rh_ipm* p, IpmStep& s, const double* rd) {
  s.a_pri = rd[rh::IR_APRI];
  s.a_dual = rd[rh::IR_ADUAL];
  s.dphi = rd[rh::IR_DPHI];
  s.theta = s.red[rh::IR_THETA];
  s.phi = s.f0 - s.mu * s.red[rh::IR_LOGSUM];
  if (p->iter == 0 && p->theta0 < 0.0) p->theta0 = s.theta;
  const double th0 = p->theta0 < 0.0 ? s.theta : p->theta0;
  s.theta_max = 1e4 * std::max(1.0, th0);
  s.theta_min = 1e-4 * std::max(1.0, th0);
  double a_min = kGammaTheta;
  if (s.dphi < 0.0) {
    a_min = std::min(a_min, kGammaPhi * s.theta / -s.dphi);
    if (s.theta <= s.theta_min)
      a_min = std::min(a_min, kDeltaSw * std::pow(s.theta, kSTheta) / std::pow(-s.dphi, kSPhi));
  }
  s.a_min = a_min * kGammaAlpha;
  s.alpha = s.a_pri;
  s.trials = 0;
}

rh_status ipm_dir_read(rh_ipm* p, IpmStep& s) {
  double rd[rh::IR_NSLOT];
  RH_TRY(read_red(p, rd, nullptr));
  ipm_dir_logic(p, s, rd);
  return RH_OK;
}

// false (and the iteration ends with RH_NOT_CONVERGED) once the step is too short
bool ipm_trial_ok(rh_ipm* p, IpmStep& s, rh_ipm_info* info) {
  if (s.alpha >= s.a_min) return true;
  fill_info(p, info, s.f0 / p->sigma_f, std::max(s.red[rh::IR_PRIM_G], s.red[rh::IR_PRIM_H]),
            s.e0, s.alpha, s.a_dual, s.delta, s.trials);
  s.done = true;
  s.code = RH_NOT_CONVERGED;
  return false;
}

rh_status ipm_trial_launch(rh_ipm* p, IpmStep& s) {
  rh_net* n = p->net;
  const auto& d = n->d;
  auto& v = p->v;
  hipStream_t st = n->stream;
  RH_HIP(rh::launch_ipm_trial(v, s.alpha, st));
  RH_HIP(rh::launch_eval(d, v.wt + v.nu, v.wt, nullptr, nullptr, false, st));
  RH_HIP(rh::launch_eval_objective(d, v.wt, v.f + 1, st));
  RH_HIP(rh::launch_ipm_stats(d, v, v.wt, v.st, 0, st));
  return RH_OK;
}

// filter acceptance of the trial point from its reductions in s.rt, s.ft;
// halves alpha if rejected
void ipm_trial_logic(rh_ipm* p, IpmStep& s, bool* accepted) {
  ++s.trials;
  const double th_t = s.rt[rh::IR_THETA];
  const double ph_t = s.ft[1] - s.mu * s.rt[rh::IR_LOGSUM];
  bool ok = std::isfinite(ph_t) && th_t <= s.theta_max;
  if (ok)
    for (const auto& e : p->filt)
      if (th_t >= e.first && ph_t >= e.second) {
        ok = false;
        break;
      }
  s.ftype = false;
  if (ok) {
    const bool switching = s.dphi < 0.0 &&
                           s.alpha * std::pow(-s.dphi, kSPhi) > kDeltaSw * std::pow(s.theta, kSTheta);
    if (switching && s.theta <= s.theta_min) {
      ok = ph_t <= s.phi + kEtaPhi * s.alpha * s.dphi;
      s.ftype = true;
    } else {
      ok = th_t <= (1.0 - kGammaTheta) * s.theta || ph_t <= s.phi - kGammaPhi * s.theta;
    }
  }
  *accepted = ok;
  if (!ok) s.alpha *= 0.5;
}

rh_status ipm_trial_accept(rh_ipm* p, IpmStep& s, bool* accepted) {
  RH_TRY(read_red(p, s.rt, s.ft));
  ipm_trial_logic(p, s, accepted);
  return RH_OK;
}

// bookkeeping of an accepted step (the update itself is launched apart)
void ipm_finish_logic(rh_ipm* p, IpmStep& s, rh_ipm_info* info) {
  if (!s.ftype) p->filt.push_back({(1.0 - kGammaTheta) * s.theta, s.phi - kGammaPhi * s.theta});
  p->iter += 1;
  fill_info(p, info, s.ft[1] / p->sigma_f, std::max(s.rt[rh::IR_PRIM_G], s.rt[rh::IR_PRIM_H]), s.e0,
            s.alpha, s.a_dual, s.delta, s.trials);
  s.done = true;
  s.code = RH_OK;
}

rh_status ipm_finish(rh_ipm* p, IpmStep& s, rh_ipm_info* info) {
  RH_HIP(rh::launch_ipm_update(p->v, s.alpha, s.a_dual, s.mu, kKappaSigma, p->net->stream));
  ipm_finish_logic(p, s, info);
  return RH_OK;
}

// Device descriptors of the batch's solvers (uploaded when the solvers
// change): copies of their IpmDev with the reductions and objective values
// redirected to batch-wide arrays, and the evaluation arguments.
rh_status ipm_batch_bind(rh_batch* b, rh_ipm* const* ipms) {
  const size_t cnt = b->nets.size();
  // solvers are told apart by their ids (a new solver may reuse the address
  // of a destroyed one)
  bool same = b->ipm_solvers.size() == cnt && b->d_ipm;
  for (size_t i = 0; same && i < cnt; ++i) same = b->ipm_solvers[i] == ipms[i]->id;
  if (same) return RH_OK;
  auto grab = [](size_t bytes, auto** out) {
    void* q = nullptr;
    if (hipMalloc(&q, bytes) != hipSuccess) return RH_ERR_OOM;
    *out = static_cast<std::remove_pointer_t<decltype(out)>>(q);
    return RH_OK;
  };
  if (!b->d_ipm) {
    RH_TRY(grab(sizeof(rh::IpmDev) * cnt, &b->d_ipm));
    RH_TRY(grab(sizeof(rh::BatchArg) * cnt, &b->d_eargs));
    RH_TRY(grab(sizeof(rh::BatchArg) * cnt, &b->d_targs));
    RH_TRY(grab(sizeof(double) * rh::kIpmSc * cnt, &b->d_sc));
    // reductions and objective values: pinned host memory that the kernels
    // write with plain stores and the host reads after a synchronise
    auto hgrab = [](size_t bytes, double** out) {
      void* q = nullptr;
      if (hipHostMalloc(&q, bytes, hipHostMallocCoherent) != hipSuccess) return RH_ERR_OOM;
      *out = static_cast<double*>(q);
      return RH_OK;
    };
    RH_TRY(hgrab(sizeof(double) * rh::IR_NSLOT * cnt, &b->d_red));
    RH_TRY(hgrab(sizeof(double) * 2 * cnt, &b->d_f));
  }
  std::vector<rh::IpmDev> dv(cnt);
  std::vector<rh::BatchArg> ea(cnt), ta(cnt);
  b->max_vec = 0;
  for (size_t i = 0; i < cnt; ++i) {
    const rh::IpmDev& v = ipms[i]->v;
    dv[i] = v;
    dv[i].red = b->d_red + rh::IR_NSLOT * i;
    dv[i].f = b->d_f + 2 * i;
    ea[i] = rh::BatchArg{};
    ea[i].x = v.w + v.nu; ea[i].u = v.w; ea[i].lam = v.lam; ea[i].y = v.y;
    ta[i] = rh::BatchArg{};
    ta[i].x = v.wt + v.nu; ta[i].u = v.wt;
    b->max_vec = std::max(b->max_vec, std::max(v.nu + v.nx, v.m));
  }
  hipStream_t st = b->stream;
  RH_HIP(hipMemcpyAsync(b->d_ipm, dv.data(), sizeof(rh::IpmDev) * cnt, hipMemcpyHostToDevice, st));
  RH_HIP(hipMemcpyAsync(b->d_eargs, ea.data(), sizeof(rh::BatchArg) * cnt, hipMemcpyHostToDevice,
                        st));
  RH_HIP(hipMemcpyAsync(b->d_targs, ta.data(), sizeof(rh::BatchArg) * cnt, hipMemcpyHostToDevice,
                        st));
  RH_HIP(hipStreamSynchronize(st));
  b->ipm_solvers.resize(cnt);
  for (size_t i = 0; i < cnt; ++i) b->ipm_solvers[i] = ipms[i]->id;
  b->h_sc.assign(size_t(rh::kIpmSc) * cnt, 0.0);
  b->h_red.assign(size_t(rh::IR_NSLOT) * cnt, 0.0);
  b->h_f.assign(2 * cnt, 0.0);
  return RH_OK;
}

void ipm_sc(rh_batch* b, size_t i, double mu, double tau, double alpha, double alpha_z,
            bool active) {
  double* q = &b->h_sc[size_t(rh::kIpmSc) * i];
  q[rh::IS_MU] = mu;
  q[rh::IS_TAU] = tau;
  q[rh::IS_ALPHA] = alpha;
  q[rh::IS_ALPHA_Z] = alpha_z;
  q[rh::IS_ACTIVE] = active ? 1.0 : 0.0;
}

// Evaluation of the active solvers at their iterates (trial = 0: with the
// Hessian, objective, grad L, full reductions) or trial points (trial = 1:
// objective and the primal reductions); scalars uploaded first.
rh_status ipm_batch_launch(rh_batch* b, int trial, bool upload_sc) {
  hipStream_t st = b->stream;
  const int cnt = int(b->nets.size());
  if (upload_sc)
    RH_HIP(hipMemcpyAsync(b->d_sc, b->h_sc.data(), sizeof(double) * b->h_sc.size(),
                          hipMemcpyHostToDevice, st));
  RH_HIP(rh::launch_batch_ipm_eval(b->d_nets, trial ? b->d_targs : b->d_eargs, b->d_ipm, b->d_sc,
                                   b->shape, trial, st));
  if (!trial)
    RH_HIP(rh::launch_ipm_batch(rh::IB_LAG_GRAD, b->d_nets, b->d_ipm, b->d_sc, cnt, b->max_vec, 0,
                                0, 0.0, st));
  RH_HIP(rh::launch_ipm_batch(rh::IB_STATS, b->d_nets, b->d_ipm, b->d_sc, cnt, b->max_vec, trial,
                              trial ? 0 : 1, 0.0, st));
  return RH_OK;
}

// all reductions (and objective values) of the batch to the host
rh_status ipm_batch_read(rh_batch* b, bool with_f) {
  RH_HIP(hipStreamSynchronize(b->stream));
  std::memcpy(b->h_red.data(), b->d_red, sizeof(double) * b->h_red.size());   // pinned host memory
  if (with_f) std::memcpy(b->h_f.data(), b->d_f, sizeof(double) * b->h_f.size());
  return RH_OK;
}

}  // namespace

extern "C" {

rh_status rh_ipm_default_options(rh_ipm_options* o) {
  if (!o) return RH_ERR_ARG;
  std::memset(o, 0, sizeof(*o));
  o->tol = 1e-6;
  o->max_iter = 200;
  o->mu_init = 0.1;
  o->obj_scale = 0.0;
  return RH_OK;
}

rh_status rh_ipm_create(rh_net* n, const rh_ipm_options* opts, const double* x0,
                        const double* u0, rh_ipm** out) {
  if (!n || !out) return RH_ERR_ARG;
  std::unique_ptr<rh_ipm> p(new (std::nothrow) rh_ipm());
  if (!p) return RH_ERR_OOM;
  static std::atomic<unsigned long long> next_id{1};
  p->id = next_id.fetch_add(1);
  p->net = n;
  if (opts) p->opt = *opts; else rh_ipm_default_options(&p->opt);
  if (!(p->opt.tol > 0.0) || p->opt.max_iter < 0 || !(p->opt.mu_init > 0.0) ||
      !(p->opt.obj_scale >= 0.0))
    return RH_ERR_ARG;
  const rh::Symbolic& s = n->s;
  auto& v = p->v;
  v.nu = s.nu;
  v.nx = s.nx;
  v.m = s.m;
  const int nw = s.nw, m = s.m, nx = s.nx, nu = s.nu;
  rh_status st_ = RH_OK;
  auto fail = [&](rh_status c) { free_ipm(p.get()); return c; };
#define IPM_TRY(expr)              \
  do {                             \
    st_ = (expr);                  \
    if (st_ != RH_OK) return fail(st_); \
  } while (0)
  IPM_TRY(setup_ipm_dev(p.get(), n, v, &p->nfin));
  IPM_TRY(ialloc(p.get(), size_t(nu) * nu, &p->K));
  IPM_TRY(ialloc(p.get(), size_t(nu) * nu, &p->Kc));
  IPM_TRY(ialloc(p.get(), nu, &p->rhs));
  hipStream_t st = n->stream;
  // initial point: the caller's, or theta = 0, Vm = 1, Pg mid-range
  if (x0 && u0) {
    if (hipMemcpyAsync(v.w, u0, sizeof(double) * nu, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(v.w + nu, x0, sizeof(double) * nx, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(RH_ERR_HIP);
  } else if (x0 || u0) {
    return fail(RH_ERR_ARG);
  } else {
    std::vector<double> w(nw, 0.0);
    for (int k = 0; k < nu; ++k)
      w[k] = s.u_kind[k] == 1 ? 1.0 : 0.5 * (n->wl[k] + n->wu[k]);
    for (int k = 0; k < nx; ++k) w[nu + k] = s.x_kind[k] == 1 ? 1.0 : 0.0;
    if (hipMemcpy(v.w, w.data(), sizeof(double) * nw, hipMemcpyHostToDevice) != hipSuccess)
      return fail(RH_ERR_HIP);
  }
  // the objective is scaled at the initial point (pushed inside the bounds)
  IPM_TRY(rh_set_objective_scale(n, 1.0));
  if (rh::launch_ipm_init_w(v, kBoundPush, kBoundFrac, st) != hipSuccess ||
      rh::launch_eval(n->d, v.w + nu, v.w, v.lam, v.y, false, st) != hipSuccess ||
      rh::launch_ipm_init_s(n->d, v, kBoundPush, kBoundFrac, st) != hipSuccess ||
      rh::launch_ipm_lag_grad(n->d, v, st) != hipSuccess ||
      rh::launch_ipm_stats(n->d, v, v.w, v.s, 1, st) != hipSuccess)
    return fail(RH_ERR_HIP);
  double red[rh::IR_NSLOT];
  IPM_TRY(read_red(p.get(), red, nullptr));
  p->sigma_f = p->opt.obj_scale > 0.0 ? p->opt.obj_scale
                                      : std::min(1.0, 100.0 / std::max(red[rh::IR_GFMAX], 1e-300));
  IPM_TRY(rh_set_objective_scale(n, p->sigma_f));
#undef IPM_TRY
  p->mu = p->opt.mu_init;
  *out = p.release();
  return RH_OK;
}

void rh_ipm_destroy(rh_ipm* p) {
  if (!p) return;
  if (p->net) {
    (void)hipStreamSynchronize(p->net->stream);
    (void)rh_set_objective_scale(p->net, 1.0);
  }
  free_ipm(p);
  delete p;
}

rh_status rh_ipm_step(rh_ipm* p, rh_ipm_info* info) {
  if (!p) return RH_ERR_ARG;
  IpmStep s;
  RH_TRY(ipm_eval_launch(p));
  RH_TRY(ipm_begin(p, s, info));
  if (s.done) return s.code;
  RH_TRY(ipm_condense_single(p));
  RH_TRY(ipm_factor(p, s, info, ipm_first_solve(p)));
  if (s.done) return s.code;
  RH_TRY(ipm_dir_launch(p, s));
  RH_TRY(ipm_dir_read(p, s));
  for (;;) {
    if (!ipm_trial_ok(p, s, info)) return s.code;
    RH_TRY(ipm_trial_launch(p, s));
    bool accepted = false;
    RH_TRY(ipm_trial_accept(p, s, &accepted));
    if (accepted) break;
  }
  return ipm_finish(p, s, info);
}

rh_status rh_ipm_batch_step(rh_batch* b, rh_ipm* const* ipms, rh_ipm_info* infos,
                            int32_t* codes) {
  if (!b || !ipms) return RH_ERR_ARG;
  const size_t cnt = b->nets.size();
  for (size_t i = 0; i < cnt; ++i)
    if (!ipms[i] || ipms[i]->net != b->nets[i]) return RH_ERR_ARG;
  RH_TRY(ipm_batch_bind(b, ipms));
  hipStream_t st = b->stream;
  std::vector<IpmStep> S(cnt);
  auto inf = [&](size_t i) { return infos ? &infos[i] : nullptr; };
  for (size_t i = 0; i < cnt; ++i) {
    rh_ipm* p = ipms[i];
    if (p->net->obj_scale != p->sigma_f) RH_TRY(rh_set_objective_scale(p->net, p->sigma_f));
  }
  RH_TRY(batch_wait_instances(b));
  RH_TRY(batch_upload(b));
  // evaluation of every solver at its iterate (one launch per kernel)
  for (size_t i = 0; i < cnt; ++i) ipm_sc(b, i, 0.0, 0.0, 0.0, 0.0, true);
  RH_TRY(ipm_batch_launch(b, 0, true));
  RH_TRY(ipm_batch_read(b, true));
  bool any = false;
  for (size_t i = 0; i < cnt; ++i) {
    std::copy_n(&b->h_red[i * rh::IR_NSLOT], rh::IR_NSLOT, S[i].red);
    std::copy_n(&b->h_f[2 * i], 2, S[i].f2);
    ipm_begin_logic(ipms[i], S[i], inf(i));
    any = any || !S[i].done;
  }
  if (any) {
    // residuals and Sigma, then one batched condensation and one batched
    // solve (delta_w = 0) for every instance (finished ones too: their
    // matrices are the solver's scratch)
    for (size_t i = 0; i < cnt; ++i) ipm_sc(b, i, S[i].mu, 0.0, 0.0, 0.0, !S[i].done);
    RH_HIP(hipMemcpyAsync(b->d_sc, b->h_sc.data(), sizeof(double) * b->h_sc.size(),
                          hipMemcpyHostToDevice, st));
    RH_HIP(rh::launch_ipm_batch(rh::IB_PREP, b->d_nets, b->d_ipm, b->d_sc, int(cnt), b->max_vec, 0,
                                0, 0.0, st));
    std::vector<rh_batch_condense_item> ci(cnt);
    std::vector<rh_batch_solve_item> si(cnt);
    for (size_t i = 0; i < cnt; ++i) {
      rh_ipm* p = ipms[i];
      auto& v = p->v;
      const int nu = v.nu;
      ci[i] = rh_batch_condense_item{};
      ci[i].x = v.w + nu; ci[i].u = v.w; ci[i].lam = v.lam; ci[i].y = v.y;
      ci[i].sig_x = v.sig_w + nu; ci[i].sig_u = v.sig_w; ci[i].sig_s = v.sig_s;
      ci[i].r = v.r; ci[i].K = p->K; ci[i].ldk = nu; ci[i].rhs = p->rhs;
      si[i] = rh_batch_solve_item{};
      si[i].K = p->K; si[i].ldk = nu; si[i].delta_w = 0.0; si[i].rhs = p->rhs;
      si[i].r = v.r; si[i].p = v.p;
    }
    RH_TRY(rh_batch_condense(b, ci.data()));
    for (size_t i = 0; i < cnt; ++i) {
      const int nu = ipms[i]->v.nu;
      RH_HIP(hipMemcpyAsync(ipms[i]->Kc, ipms[i]->K, sizeof(double) * size_t(nu) * nu,
                            hipMemcpyDeviceToDevice, st));
    }
    std::vector<int32_t> stt(cnt, RH_OK);
    const rh_status bs = rh_batch_solve(b, si.data(), stt.data());
    if (bs < 0 && bs != RH_ERR_STATE) return bs;
    // inertia-correction retries per solver (the batch stream has drained)
    for (size_t i = 0; i < cnt; ++i)
      if (!S[i].done) RH_TRY(ipm_factor(ipms[i], S[i], inf(i), rh_status(stt[i])));
    RH_TRY(batch_wait_instances(b));
    // bound-multiplier steps and the largest steps to the boundary
    for (size_t i = 0; i < cnt; ++i)
      ipm_sc(b, i, S[i].mu, std::max(kTauMin, 1.0 - S[i].mu), 0.0, 0.0, !S[i].done);
    RH_HIP(hipMemcpyAsync(b->d_sc, b->h_sc.data(), sizeof(double) * b->h_sc.size(),
                          hipMemcpyHostToDevice, st));
    RH_HIP(rh::launch_ipm_batch(rh::IB_DIR, b->d_nets, b->d_ipm, b->d_sc, int(cnt), b->max_vec, 0,
                                0, 0.0, st));
    RH_TRY(ipm_batch_read(b, false));
    for (size_t i = 0; i < cnt; ++i)
      if (!S[i].done) ipm_dir_logic(ipms[i], S[i], &b->h_red[i * rh::IR_NSLOT]);
    // filter line searches in lockstep: one trial per unfinished solver per round
    std::vector<char> acc(cnt, 0);
    for (;;) {
      bool pending = false;
      for (size_t i = 0; i < cnt; ++i) {
        const bool go = !S[i].done && !acc[i] && ipm_trial_ok(ipms[i], S[i], inf(i));
        ipm_sc(b, i, S[i].mu, 0.0, S[i].alpha, 0.0, go);
        pending = pending || go;
      }
      if (!pending) break;
      RH_HIP(hipMemcpyAsync(b->d_sc, b->h_sc.data(), sizeof(double) * b->h_sc.size(),
                            hipMemcpyHostToDevice, st));
      RH_HIP(rh::launch_ipm_batch(rh::IB_TRIAL, b->d_nets, b->d_ipm, b->d_sc, int(cnt),
                                  b->max_vec, 0, 0, 0.0, st));
      RH_TRY(ipm_batch_launch(b, 1, false));
      RH_TRY(ipm_batch_read(b, true));
      for (size_t i = 0; i < cnt; ++i)
        if (b->h_sc[size_t(rh::kIpmSc) * i + rh::IS_ACTIVE] != 0.0) {
          std::copy_n(&b->h_red[i * rh::IR_NSLOT], rh::IR_NSLOT, S[i].rt);
          std::copy_n(&b->h_f[2 * i], 2, S[i].ft);
          bool ok = false;
          ipm_trial_logic(ipms[i], S[i], &ok);
          acc[i] = ok ? 1 : 0;
        }
    }
    // updates of the accepted steps
    for (size_t i = 0; i < cnt; ++i)
      ipm_sc(b, i, S[i].mu, 0.0, S[i].alpha, S[i].a_dual, !S[i].done && acc[i]);
    RH_HIP(hipMemcpyAsync(b->d_sc, b->h_sc.data(), sizeof(double) * b->h_sc.size(),
                          hipMemcpyHostToDevice, st));
    RH_HIP(rh::launch_ipm_batch(rh::IB_UPDATE, b->d_nets, b->d_ipm, b->d_sc, int(cnt), b->max_vec,
                                0, 0, kKappaSigma, st));
    for (size_t i = 0; i < cnt; ++i)
      if (!S[i].done && acc[i]) ipm_finish_logic(ipms[i], S[i], inf(i));
    RH_HIP(hipStreamSynchronize(st));
  }
  if (codes)
    for (size_t i = 0; i < cnt; ++i) codes[i] = S[i].code;
  return RH_OK;
}

rh_status rh_ipm_solve(rh_ipm* p, rh_ipm_info* info) {
  if (!p) return RH_ERR_ARG;
  rh_ipm_info last{};
  for (;;) {
    rh_status c = rh_ipm_step(p, &last);
    if (c != RH_OK) {
      if (info) *info = last;
      return c;
    }
    if (last.converged) break;
  }
  if (info) *info = last;
  return RH_OK;
}

rh_status rh_ipm_outputs(const rh_ipm* p, double* pg, double* vm, double* f) {
  if (!p) return RH_ERR_ARG;
  rh_net* n = p->net;
  RH_HIP(rh::launch_opf_outputs(n->d, p->v, 1.0 / p->sigma_f, pg, vm, f, n->stream));
  return RH_OK;
}

rh_status rh_ipm_backward(rh_ipm* p, const double* dpg, const double* dvm, const double* df,
                          double* gpd, double* gqd, double* xi) {
  if (!p || !gpd || !gqd) return RH_ERR_ARG;
  if (!p->converged) return RH_ERR_STATE;
  rh_net* n = p->net;
  auto& v = p->v;
  const auto& d = n->d;
  hipStream_t st = n->stream;
  const int nu = v.nu;
  if (n->obj_scale != p->sigma_f) RH_TRY(rh_set_objective_scale(n, p->sigma_f));
  {
    PhaseScope ps(n, RH_PHASE_EVAL);
    RH_HIP(rh::launch_eval(d, v.w + nu, v.w, v.lam, v.y, true, st));
  }
  // Sigma of the final iterate (the residuals prep writes are replaced by the
  // adjoint right-hand side)
  RH_HIP(rh::launch_ipm_prep(d, v, p->mu, st));
  RH_HIP(rh::launch_adjoint_rhs(d, v, 1.0 / p->sigma_f, dpg, dvm, df, v.r, st));
  RH_TRY(condense_evaluated(n, v.sig_w + nu, v.sig_w, v.sig_s, v.r, p->K, nu, p->rhs));
  const rh_status code = rh_solve_condensed_kkt(n, p->K, nu, 0.0, p->rhs, v.r, v.p, nullptr);
  if (code != RH_OK) return code;     // no gradient from unusable factors
  RH_HIP(rh::launch_adjoint_grad(d, v, v.p, gpd, gqd, st));
  if (xi) {
    const size_t np = size_t(nu) + 2 * size_t(v.nx) + 2 * size_t(v.m);
    RH_HIP(hipMemcpyAsync(xi, v.p, sizeof(double) * np, hipMemcpyDeviceToDevice, st));
  }
  return code;
}

rh_status rh_ipm_batch_backward(rh_batch* b, rh_ipm* const* ipms, const double* const* dpg,
                                const double* const* dvm, const double* const* df,
                                double* const* gpd, double* const* gqd, int32_t* codes) {
  if (!b || !ipms || !gpd || !gqd) return RH_ERR_ARG;
  const size_t cnt = b->nets.size();
  for (size_t i = 0; i < cnt; ++i) {
    if (!ipms[i] || ipms[i]->net != b->nets[i] || !gpd[i] || !gqd[i]) return RH_ERR_ARG;
    if (!ipms[i]->converged) return RH_ERR_STATE;
  }
  RH_TRY(ipm_batch_bind(b, ipms));
  hipStream_t st = b->stream;
  for (size_t i = 0; i < cnt; ++i) {
    rh_ipm* p = ipms[i];
    if (p->net->obj_scale != p->sigma_f) RH_TRY(rh_set_objective_scale(p->net, p->sigma_f));
  }
  RH_TRY(batch_wait_instances(b));
  RH_TRY(batch_upload(b));
  // Sigma of each final iterate, the adjoint right-hand sides, then one
  // batched condensation and solve
  for (size_t i = 0; i < cnt; ++i) ipm_sc(b, i, ipms[i]->mu, 0.0, 0.0, 0.0, true);
  RH_HIP(hipMemcpyAsync(b->d_sc, b->h_sc.data(), sizeof(double) * b->h_sc.size(),
                        hipMemcpyHostToDevice, st));
  RH_HIP(rh::launch_ipm_batch(rh::IB_PREP, b->d_nets, b->d_ipm, b->d_sc, int(cnt), b->max_vec, 0,
                              0, 0.0, st));
  std::vector<rh_batch_condense_item> ci(cnt);
  std::vector<rh_batch_solve_item> si(cnt);
  for (size_t i = 0; i < cnt; ++i) {
    rh_ipm* p = ipms[i];
    auto& v = p->v;
    const int nu = v.nu;
    RH_HIP(rh::launch_adjoint_rhs(p->net->d, v, 1.0 / p->sigma_f, dpg ? dpg[i] : nullptr,
                                  dvm ? dvm[i] : nullptr, df ? df[i] : nullptr, v.r, st));
    ci[i] = rh_batch_condense_item{};
    ci[i].x = v.w + nu; ci[i].u = v.w; ci[i].lam = v.lam; ci[i].y = v.y;
    ci[i].sig_x = v.sig_w + nu; ci[i].sig_u = v.sig_w; ci[i].sig_s = v.sig_s;
    ci[i].r = v.r; ci[i].K = p->K; ci[i].ldk = nu; ci[i].rhs = p->rhs;
    si[i] = rh_batch_solve_item{};
    si[i].K = p->K; si[i].ldk = nu; si[i].delta_w = 0.0; si[i].rhs = p->rhs;
    si[i].r = v.r; si[i].p = v.p;
  }
  RH_TRY(rh_batch_condense(b, ci.data()));
  std::vector<int32_t> stt(cnt, RH_OK);
  const rh_status bs = rh_batch_solve(b, si.data(), stt.data());
  if (bs < 0 && bs != RH_ERR_STATE) return bs;
  for (size_t i = 0; i < cnt; ++i) {
    if (stt[i] != RH_OK) continue;     // no gradient from unusable factors
    rh_ipm* p = ipms[i];
    RH_HIP(rh::launch_adjoint_grad(p->net->d, p->v, p->v.p, gpd[i], gqd[i], st));
  }
  RH_HIP(hipStreamSynchronize(st));
  if (codes)
    for (size_t i = 0; i < cnt; ++i) codes[i] = stt[i];
  return RH_OK;
}

rh_status rh_ipm_get_state(const rh_ipm* p, double* x, double* u, double* s, double* lam,
                           double* y) {
  if (!p) return RH_ERR_ARG;
  const auto& v = p->v;
  hipStream_t st = p->net->stream;
  if (u) RH_HIP(hipMemcpyAsync(u, v.w, sizeof(double) * v.nu, hipMemcpyDeviceToDevice, st));
  if (x) RH_HIP(hipMemcpyAsync(x, v.w + v.nu, sizeof(double) * v.nx, hipMemcpyDeviceToDevice, st));
  if (s) RH_HIP(hipMemcpyAsync(s, v.s, sizeof(double) * v.m, hipMemcpyDeviceToDevice, st));
  if (lam) RH_HIP(hipMemcpyAsync(lam, v.lam, sizeof(double) * v.nx, hipMemcpyDeviceToDevice, st));
  if (y) RH_HIP(hipMemcpyAsync(y, v.y, sizeof(double) * v.m, hipMemcpyDeviceToDevice, st));
  return RH_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Newton-Raphson power flow and the reduce-then-linearize driver (Algorithm 2)
// ---------------------------------------------------------------------------
namespace {

constexpr double kPfTol = 1e-10;   // projection tolerance (the paper's)
constexpr int kPfMaxIter = 20;

// Newton-Raphson on g(x, u) = 0 in place: every iteration evaluates g, reads
// max |g| (one scalar), refactorises G_x and solves x -= G_x^{-1} g with the
// condensation's sweeps. iters: Newton steps taken; res: the last max |g|.
rh_status newton_pf(rh_net* n, const double* u, double* x, double tol, int max_iter, int* iters,
                    double* res) {
  const auto& d = n->d;
  hipStream_t st = n->stream;
  if (!n->pf_scal)
    RH_HIP(hipHostMalloc(reinterpret_cast<void**>(&n->pf_scal), 4 * sizeof(double),
                         hipHostMallocCoherent));
  for (int k = 0;; ++k) {
    RH_HIP(rh::launch_eval(d, x, u, nullptr, nullptr, false, st));
    RH_HIP(rh::launch_absmax(d.dst + d.d_g, d.nx, n->pf_scal, st));
    RH_HIP(hipStreamSynchronize(st));
    const double gm = n->pf_scal[0];   // written by the reduction kernel
    if (iters) *iters = k;
    if (res) *res = gm;
    if (gm <= tol) return RH_OK;
    if (k >= max_iter || !std::isfinite(gm)) return RH_NOT_CONVERGED;
    RH_HIP(rh::launch_refactor(d, st));
    RH_HIP(rh::launch_gx_solve(d, n->width, n->lds, false, d.dst + d.d_g, x, -1.0, true, st));
  }
}

}  // namespace

struct rh_redlin {
  rh_net* net = nullptr;
  rh_ipm_options opt{};
  rh::IpmDev v{};       // full space: w = [u; x], lambda (adjoint), s -> sr, y -> yr
  rh::IpmDev rv{};      // reduced variables: w = u, s = s_r, y = y_r (nx = 0)
  rh::RedLinDev R{};
  std::vector<void*> allocs;
  std::vector<void*> hallocs;   // pinned host memory (the reduction slots, objective values)
  double *K = nullptr, *Kc = nullptr, *rhs = nullptr, *adj = nullptr, *scal = nullptr;
  double mu = 0.1, delta_last = 0.0, theta0 = -1.0, sigma_f = 1.0;
  std::vector<std::pair<double, double>> filt;
  long iter = 0;
  int nfin = 0;
  bool converged = false;
};

namespace {

double redlin_error(const rh_redlin* p, const double* red, double mu) {
  const double sd = std::max(kSMax, (red[rh::IR_LYSUM] + red[rh::IR_ZSUM]) /
                                        std::max(1, p->R.mr + p->nfin)) / kSMax;
  const double sc = std::max(kSMax, red[rh::IR_ZSUM] / std::max(1, p->nfin)) / kSMax;
  const double ed = std::max(red[rh::IR_DUAL_W], red[rh::IR_DUAL_S]) / sd;
  const double ep = red[rh::IR_PRIM_H];
  const double ec =
      p->nfin ? std::max(red[rh::IR_DZ_MAX] - mu, mu - red[rh::IR_DZ_MIN]) / sc : 0.0;
  return std::max(ed, std::max(ep, ec));
}

rh_status redlin_read(rh_redlin* p, double* red, double* f) {
  RH_HIP(hipStreamSynchronize(p->net->stream));
  std::memcpy(red, p->R.red, sizeof(double) * rh::IR_NSLOT);   // pinned host memory
  if (f) std::memcpy(f, p->v.f, sizeof(double) * 2);
  return RH_OK;
}

// Derivatives at the current (projected) point: adjoint lambda =
// -G_x^{-T}(grad_x f + A_x^T y_h - y_x), then the Hessian of
// f + lambda^T g + y_h^T h, grad L (whose u part is the reduced gradient),
// the objective and the reductions.
rh_status redlin_derivatives(rh_redlin* p, double* red, double* f) {
  rh_net* n = p->net;
  const auto& d = n->d;
  auto& v = p->v;
  hipStream_t st = n->stream;
  const int nu = v.nu;
  {
    PhaseScope ps(n, RH_PHASE_EVAL);
    RH_HIP(rh::launch_fill(v.lam, v.nx, 0.0, st));
    RH_HIP(rh::launch_eval(d, v.w + nu, v.w, nullptr, nullptr, false, st));
    RH_HIP(rh::launch_ipm_lag_grad(d, v, st));
    RH_HIP(rh::launch_redlin_adj_rhs(v, p->R, p->adj, st));
  }
  {
    PhaseScope ps(n, RH_PHASE_REFACTOR);
    RH_HIP(rh::launch_refactor(d, st));
    RH_HIP(rh::launch_gx_solve(d, n->width, n->lds, true, p->adj, v.lam, 1.0, false, st));
  }
  {
    PhaseScope ps(n, RH_PHASE_EVAL);
    RH_HIP(rh::launch_eval(d, v.w + nu, v.w, v.lam, v.y, true, st));
    RH_HIP(rh::launch_ipm_lag_grad(d, v, st));
    RH_HIP(rh::launch_eval_objective(d, v.w, v.f, st));
    RH_HIP(rh::launch_redlin_stats(d, v, p->R, v.w, p->R.sr, 1, st));
  }
  return redlin_read(p, red, f);
}

void redlin_info(const rh_redlin* p, rh_ipm_info* info, double obj, double inf_pr, double err,
                 double alpha, double alpha_z, double delta, long trials, long pf) {
  if (!info) return;
  std::memset(info, 0, sizeof(*info));
  info->iter = p->iter;
  info->obj = obj;
  info->inf_pr = inf_pr;
  info->err = err;
  info->mu = p->mu;
  info->alpha_pr = alpha;
  info->alpha_du = alpha_z;
  info->delta_w = delta;
  info->ls_trials = trials;
  info->obj_scale = p->sigma_f;
  info->converged = p->converged ? 1 : 0;
  info->pf_iters = int32_t(pf);
}

}  // namespace

extern "C" {

rh_status rh_power_flow(rh_net* n, const double* u, double* x, double tol, int32_t max_iter,
                        int32_t* iters, double* residual) {
  if (!n || !u || !x || !(tol > 0.0) || max_iter < 0) return RH_ERR_ARG;
  int k = 0;
  double res = 0.0;
  rh_status c;
  {
    PhaseScope ps(n, RH_PHASE_PROJECT);
    c = newton_pf(n, u, x, tol, max_iter, &k, &res);
  }
  if (iters) *iters = k;
  if (residual) *residual = res;
  return c;
}

rh_status rh_redlin_create(rh_net* n, const rh_ipm_options* opts, const double* x0,
                           const double* u0, rh_redlin** out) {
  if (!n || !out) return RH_ERR_ARG;
  std::unique_ptr<rh_redlin> p(new (std::nothrow) rh_redlin());
  if (!p) return RH_ERR_OOM;
  p->net = n;
  if (opts) p->opt = *opts; else rh_ipm_default_options(&p->opt);
  if (!(p->opt.tol > 0.0) || p->opt.max_iter < 0 || !(p->opt.mu_init > 0.0) ||
      !(p->opt.obj_scale >= 0.0))
    return RH_ERR_ARG;
  if ((x0 == nullptr) != (u0 == nullptr)) return RH_ERR_ARG;
  rh_status st_ = RH_OK;
  auto fail = [&](rh_status c) { free_ipm(p.get()); return c; };
#define RL_TRY(expr)               \
  do {                             \
    st_ = (expr);                  \
    if (st_ != RH_OK) return fail(st_); \
  } while (0)
  auto& v = p->v;
  auto& R = p->R;
  int nfin_full = 0;
  RL_TRY(setup_ipm_dev(p.get(), n, v, &nfin_full));
  const rh::Symbolic& s = n->s;
  const int nu = s.nu, nx = s.nx, m = s.m;
  // bounded states and the slack bounds of h_r = [h; -x_b]
  std::vector<int> xb, xbi(nx, -1);
  for (int k = 0; k < nx; ++k)
    if (std::isfinite(n->wl[nu + k]) || std::isfinite(n->wu[nu + k])) {
      xbi[k] = int(xb.size());
      xb.push_back(k);
    }
  std::vector<double> rsl(n->sl), rsu(n->su);
  for (int k : xb) {
    rsl.push_back(n->wl[nu + k]);
    rsu.push_back(n->wu[nu + k]);
  }
  R.m = m;
  R.nxb = int(xb.size());
  R.mr = m + R.nxb;
  const int mr = R.mr;
  RL_TRY(iupload(p.get(), xb, &R.xb));
  RL_TRY(iupload(p.get(), xbi, &R.xbi));
  RL_TRY(iupload(p.get(), rsl, &R.rsl));
  RL_TRY(iupload(p.get(), rsu, &R.rsu));
  RL_TRY(ialloc(p.get(), mr, &R.sr));
  RL_TRY(ialloc(p.get(), mr, &R.yr));
  RL_TRY(ialloc(p.get(), mr, &R.zsl));
  RL_TRY(ialloc(p.get(), mr, &R.zsu));
  RL_TRY(ialloc(p.get(), size_t(nu) + 2 * size_t(mr), &R.rp));
  RL_TRY(ialloc(p.get(), mr, &R.pzsl));
  RL_TRY(ialloc(p.get(), mr, &R.pzsu));
  RL_TRY(ialloc(p.get(), mr, &R.st));
  RL_TRY(ialloc(p.get(), nu, &R.zero));
  RL_TRY(halloc(p.get(), rh::IR_NSLOT, &R.red));
  RL_TRY(ialloc(p.get(), size_t(nu) * nu, &p->K));
  RL_TRY(ialloc(p.get(), size_t(nu) * nu, &p->Kc));
  RL_TRY(ialloc(p.get(), nu, &p->rhs));
  RL_TRY(ialloc(p.get(), nx, &p->adj));
  RL_TRY(halloc(p.get(), 4, &p->scal));   // read by the host after each direction
  v.s = R.sr;            // the h rows' slacks and multipliers lead s_r, y_r
  v.y = R.yr;
  p->nfin = 0;
  for (int k = 0; k < nu; ++k)
    p->nfin += (std::isfinite(n->wl[k]) ? 1 : 0) + (std::isfinite(n->wu[k]) ? 1 : 0);
  for (int j = 0; j < mr; ++j)
    p->nfin += (std::isfinite(rsl[j]) ? 1 : 0) + (std::isfinite(rsu[j]) ? 1 : 0);
  auto& rv = p->rv;
  rv.nu = nu;
  rv.nx = 0;
  rv.m = mr;
  rv.wl = v.wl;
  rv.wu = v.wu;
  rv.sl = R.rsl;
  rv.su = R.rsu;
  rv.w = v.w;
  rv.s = R.sr;
  rv.y = R.yr;
  rv.zl = v.zl;
  rv.zu = v.zu;
  rv.zsl = R.zsl;
  rv.zsu = R.zsu;
  rv.gf = R.zero;
  rv.p = R.rp;
  rv.pzl = v.pzl;
  rv.pzu = v.pzu;
  rv.pzsl = R.pzsl;
  rv.pzsu = R.pzsu;
  rv.wt = v.wt;
  rv.st = R.st;
  rv.red = R.red;
  rv.f = v.f;
  hipStream_t st = n->stream;
  if (rh::launch_fill(R.zero, nu, 0.0, st) != hipSuccess) return fail(RH_ERR_HIP);
  // initial point: the caller's, or theta = 0, Vm = 1, Pg mid-range
  if (x0) {
    if (hipMemcpyAsync(v.w, u0, sizeof(double) * nu, hipMemcpyDeviceToDevice, st) != hipSuccess ||
        hipMemcpyAsync(v.w + nu, x0, sizeof(double) * nx, hipMemcpyDeviceToDevice, st) != hipSuccess)
      return fail(RH_ERR_HIP);
  } else {
    std::vector<double> w(s.nw, 0.0);
    for (int k = 0; k < nu; ++k)
      w[k] = s.u_kind[k] == 1 ? 1.0 : 0.5 * (n->wl[k] + n->wu[k]);
    for (int k = 0; k < nx; ++k) w[nu + k] = s.x_kind[k] == 1 ? 1.0 : 0.0;
    if (hipMemcpy(v.w, w.data(), sizeof(double) * s.nw, hipMemcpyHostToDevice) != hipSuccess)
      return fail(RH_ERR_HIP);
  }
  RL_TRY(rh_set_objective_scale(n, 1.0));
  // controls pushed inside their bounds (multipliers 1, y_r = 0), then the
  // state projected onto g = 0
  if (rh::launch_ipm_init_w(rv, kBoundPush, kBoundFrac, st) != hipSuccess) return fail(RH_ERR_HIP);
  int k = 0;
  RL_TRY(newton_pf(n, v.w, v.w + nu, kPfTol, kPfMaxIter, &k, nullptr));
  // objective scale at the projected point; slacks s_r = [-h; x_b] pushed inside
  if (rh::launch_fill(v.lam, nx, 0.0, st) != hipSuccess ||
      rh::launch_ipm_lag_grad(n->d, v, st) != hipSuccess ||
      rh::launch_redlin_init_s(n->d, v, R, kBoundPush, kBoundFrac, st) != hipSuccess ||
      rh::launch_redlin_stats(n->d, v, R, v.w, R.sr, 1, st) != hipSuccess)
    return fail(RH_ERR_HIP);
  double red[rh::IR_NSLOT];
  RL_TRY(redlin_read(p.get(), red, nullptr));
  p->sigma_f = p->opt.obj_scale > 0.0 ? p->opt.obj_scale
                                      : std::min(1.0, 100.0 / std::max(red[rh::IR_GFMAX], 1e-300));
  RL_TRY(rh_set_objective_scale(n, p->sigma_f));
#undef RL_TRY
  p->mu = p->opt.mu_init;
  *out = p.release();
  return RH_OK;
}

void rh_redlin_destroy(rh_redlin* p) {
  if (!p) return;
  if (p->net) {
    (void)hipStreamSynchronize(p->net->stream);
    (void)rh_set_objective_scale(p->net, 1.0);
  }
  free_ipm(p);
  delete p;
}

rh_status rh_redlin_step(rh_redlin* p, rh_ipm_info* info) {
  if (!p) return RH_ERR_ARG;
  rh_net* n = p->net;
  if (n->obj_scale != p->sigma_f) RH_TRY(rh_set_objective_scale(n, p->sigma_f));
  auto& v = p->v;
  auto& R = p->R;
  const auto& d = n->d;
  hipStream_t st = n->stream;
  const int nu = v.nu, nx = v.nx;
  double red[rh::IR_NSLOT], f2[2];
  RH_TRY(redlin_derivatives(p, red, f2));
  const double f0 = f2[0];
  const double e0 = redlin_error(p, red, 0.0);
  if (e0 <= p->opt.tol) {
    p->converged = true;
    redlin_info(p, info, f0 / p->sigma_f, red[rh::IR_PRIM_H], e0, 0.0, 0.0, 0.0, 0, 0);
    return RH_OK;
  }
  if (p->iter >= p->opt.max_iter) {
    redlin_info(p, info, f0 / p->sigma_f, red[rh::IR_PRIM_H], e0, 0.0, 0.0, 0.0, 0, 0);
    return RH_NOT_CONVERGED;
  }
  for (int k = 0; k < 10; ++k) {
    if (redlin_error(p, red, p->mu) > kKappaEps * p->mu) break;
    const double nm = std::max(p->opt.tol / 10.0, std::min(kKappaMu * p->mu, std::pow(p->mu, kThetaMu)));
    if (nm == p->mu) break;
    p->mu = nm;
    p->filt.clear();
  }
  const double mu = p->mu;
  // the reduced KKT system through the full-space condensation
  RH_HIP(rh::launch_redlin_prep(d, v, R, mu, st));
  RH_TRY(condense_evaluated(n, v.sig_w + nu, v.sig_w, v.sig_s, v.r, p->K, nu, p->rhs, p->Kc));
  double delta = 0.0;
  rh_status code = rh_solve_condensed_kkt(n, p->K, nu, 0.0, p->rhs, v.r, v.p, nullptr);
  if (code == RH_NOT_POSDEF) {
    delta = p->delta_last == 0.0 ? kDelta0 : std::max(kDeltaMin, kKwMinus * p->delta_last);
    for (;;) {
      RH_HIP(hipMemcpyAsync(p->K, p->Kc, sizeof(double) * size_t(nu) * nu,
                            hipMemcpyDeviceToDevice, st));
      code = rh_solve_condensed_kkt(n, p->K, nu, delta, p->rhs, v.r, v.p, nullptr);
      if (code != RH_NOT_POSDEF) break;
      delta *= p->delta_last == 0.0 ? kKwPlusBar : kKwPlus;
      if (delta > kDeltaMax) {
        redlin_info(p, info, f0 / p->sigma_f, red[rh::IR_PRIM_H], e0, 0.0, 0.0, delta, 0, 0);
        return RH_NOT_CONVERGED;
      }
    }
    p->delta_last = delta;
  }
  if (code < 0) return code;
  // reduced step, bound-multiplier steps, largest steps to the boundary
  const double tau = std::max(kTauMin, 1.0 - mu);
  RH_HIP(rh::launch_redlin_pack(v, R, mu, p->scal, st));
  RH_HIP(rh::launch_ipm_dir(p->rv, mu, tau, st));
  double rd[rh::IR_NSLOT], dphi_f = 0.0;
  RH_TRY(redlin_read(p, rd, nullptr));   // also drains the stream for p->scal (pinned)
  dphi_f = p->scal[0];
  const double a_pri = rd[rh::IR_APRI], a_dual = rd[rh::IR_ADUAL];
  const double dphi = rd[rh::IR_DPHI] + dphi_f;
  const double theta = red[rh::IR_THETA];
  const double phi = f0 - mu * red[rh::IR_LOGSUM];
  if (p->iter == 0 && p->theta0 < 0.0) p->theta0 = theta;
  const double th0 = p->theta0 < 0.0 ? theta : p->theta0;
  const double theta_max = 1e4 * std::max(1.0, th0), theta_min = 1e-4 * std::max(1.0, th0);
  double a_min = kGammaTheta;
  if (dphi < 0.0) {
    a_min = std::min(a_min, kGammaPhi * theta / -dphi);
    if (theta <= theta_min)
      a_min = std::min(a_min, kDeltaSw * std::pow(theta, kSTheta) / std::pow(-dphi, kSPhi));
  }
  a_min *= kGammaAlpha;
  double alpha = a_pri;
  long trials = 0, pf = 0;
  bool ftype = false;
  double rt[rh::IR_NSLOT], ft[2];
  for (;;) {
    if (alpha < a_min) {
      redlin_info(p, info, f0 / p->sigma_f, red[rh::IR_PRIM_H], e0, alpha, a_dual, delta, trials,
                  pf);
      return RH_NOT_CONVERGED;
    }
    // trial point: controls and slacks along the step, the state projected
    // from its linearised step
    RH_HIP(rh::launch_ipm_trial(p->rv, alpha, st));
    RH_HIP(rh::launch_redlin_trial_x(v, alpha, st));
    int k = 0;
    rh_status pc;
    {
      PhaseScope ps(n, RH_PHASE_PROJECT);
      pc = newton_pf(n, v.wt, v.wt + nu, kPfTol, kPfMaxIter, &k, nullptr);
    }
    if (pc < 0) return pc;
    ++trials;
    pf += k;
    bool ok = pc == RH_OK;
    ftype = false;
    if (ok) {
      RH_HIP(rh::launch_eval_objective(d, v.wt, v.f + 1, st));
      RH_HIP(rh::launch_redlin_stats(d, v, R, v.wt, R.st, 0, st));
      RH_TRY(redlin_read(p, rt, ft));
      const double th_t = rt[rh::IR_THETA];
      const double ph_t = ft[1] - mu * rt[rh::IR_LOGSUM];
      ok = std::isfinite(ph_t) && th_t <= theta_max;
      if (ok)
        for (const auto& e : p->filt)
          if (th_t >= e.first && ph_t >= e.second) {
            ok = false;
            break;
          }
      if (ok) {
        const bool switching =
            dphi < 0.0 && alpha * std::pow(-dphi, kSPhi) > kDeltaSw * std::pow(theta, kSTheta);
        if (switching && theta <= theta_min) {
          ok = ph_t <= phi + kEtaPhi * alpha * dphi;
          ftype = true;
        } else {
          ok = th_t <= (1.0 - kGammaTheta) * theta || ph_t <= phi - kGammaPhi * theta;
        }
      }
    }
    if (ok) break;
    alpha *= 0.5;
  }
  if (!ftype) p->filt.push_back({(1.0 - kGammaTheta) * theta, phi - kGammaPhi * theta});
  RH_HIP(rh::launch_ipm_update(p->rv, alpha, a_dual, mu, kKappaSigma, st));
  RH_HIP(hipMemcpyAsync(v.w + nu, v.wt + nu, sizeof(double) * nx, hipMemcpyDeviceToDevice, st));
  p->iter += 1;
  redlin_info(p, info, ft[1] / p->sigma_f, rt[rh::IR_PRIM_H], e0, alpha, a_dual, delta, trials, pf);
  return RH_OK;
}

rh_status rh_redlin_solve(rh_redlin* p, rh_ipm_info* info) {
  if (!p) return RH_ERR_ARG;
  rh_ipm_info last{};
  for (;;) {
    rh_status c = rh_redlin_step(p, &last);
    if (c != RH_OK) {
      if (info) *info = last;
      return c;
    }
    if (last.converged) break;
  }
  if (info) *info = last;
  return RH_OK;
}

rh_status rh_redlin_get_state(const rh_redlin* p, double* x, double* u, double* s, double* lam,
                              double* y) {
  if (!p) return RH_ERR_ARG;
  const auto& v = p->v;
  hipStream_t st = p->net->stream;
  const size_t mr = size_t(p->R.mr);
  if (u) RH_HIP(hipMemcpyAsync(u, v.w, sizeof(double) * v.nu, hipMemcpyDeviceToDevice, st));
  if (x) RH_HIP(hipMemcpyAsync(x, v.w + v.nu, sizeof(double) * v.nx, hipMemcpyDeviceToDevice, st));
  if (s) RH_HIP(hipMemcpyAsync(s, p->R.sr, sizeof(double) * mr, hipMemcpyDeviceToDevice, st));
  if (lam) RH_HIP(hipMemcpyAsync(lam, v.lam, sizeof(double) * v.nx, hipMemcpyDeviceToDevice, st));
  if (y) RH_HIP(hipMemcpyAsync(y, p->R.yr, sizeof(double) * mr, hipMemcpyDeviceToDevice, st));
  return RH_OK;
}

rh_status rh_redlin_dims(const rh_redlin* p, int64_t* mr, int64_t* nxb) {
  if (!p) return RH_ERR_ARG;
  if (mr) *mr = p->R.mr;
  if (nxb) *nxb = p->R.nxb;
  return RH_OK;
}

}  // extern "C"
