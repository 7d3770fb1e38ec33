// Device-side view of one analysed network and the launch wrappers of the
// condensation hot path. All pointers are HIP device memory owned by rh_net.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

namespace rh {

// Read-only descriptor arrays of the batched launches (written by the host
// before the launch, never by a kernel) are read through the constant
// address space: pointers loaded from constant memory are known to address
// global memory, so the kernels use global rather than flat loads and
// stores through them (a flat load also holds up every wait for LDS).
template <class T>
__device__ __forceinline__ const T& cst(const T* p, int i) {
  return *(const T*)((const __attribute__((address_space(4))) T*)p + i);
}

struct DevSweep {
  int nlev = 0;
  const int* lev_ptr = nullptr;   // nlev + 1: level sets (refactorisation schedule)
  const int* rows = nullptr;      // nx: row per level-ordered slot
  // condensation schedule: kSweepMeta ints per step {step index in
  // DevNet::lblk, log2 lanes per row, 0, 0}, then the idle step
  int nstep = 0;
  const int* meta = nullptr;
  // the same steps as NW lists of ngrp + 1 entries (wave after wave), for
  // work-groups of NW waves: [0] NW = kCondWaves, [1] NW = kCondWavesWide
  int ngrp[2] = {0, 0};
  const int* gmeta[2] = {nullptr, nullptr};
  int unit = 0;                   // 1: unit diagonal (L and L^T sweeps)
};

struct DevNet {
  int nb, nl, ng, nx, nu, m, nw, nlim, ref, ref_gen;
  // 1: the condensation's panel fills the LDS, so the kernels read the sweep
  // metadata from global memory instead of staging it (one column per
  // work-group)
  int meta_global;
  int cond_nw;   // waves per condensation work-group (1, kCondWaves, kCondWavesWide)
  // with several waves: bit k set = sweep k (L, U, U^T, L^T) runs on all of
  // them (same-level steps spread over the waves), else on one
  int sweep_grouped;
  double base, c2_ref, c1_ref, cost_rank1;
  const double *c2, *c1, *c0;
  const int* pg_u;
  // lines and buses
  const int *lf, *lt;
  const double *gff, *bff, *gft, *bft;
  const int *th_nat, *vmx_nat, *vmu;
  const int *line_w, *line_wsrc;
  const int *ref_lines, *ref_ends;
  int n_ref_lines;
  const int *perm, *iperm;
  // LU and refactorisation
  int nnz_lu, max_row;
  const int *lu_ptr, *lu_col, *lu_diag;
  const int *rf_kptr, *rf_src, *rf_dst;
  const int *rf_piv, *rf_dst_local;
  int max_row_ops, max_row_lower, rf_groups;   // rf_groups rows factored at once
  const int *rf_rows;             // rows in L-level order (= sl.rows)
  const int *rf_lev_ptr;
  int rf_nlev;
  DevSweep sl, su, sut, slt;
  // G_u, A, K patterns
  int nnz_gu, nnz_a, nnz_k;
  const int *gu_ptr, *gu_col, *gucsc_ptr, *gucsc_row, *gucsc_from;
  const int *a_ptr, *a_col, *acsc_ptr, *acsc_row, *acsc_from;
  const int *k_ptr, *k_col;
  const int *kg_hl_ptr, *kg_hl_idx, *kg_ata_ptr, *kg_a1, *kg_a2, *kg_row, *kg_diag;
  const int* sig_map;
  // Condensation records for the launch width (rh::CondenseRecords): sweep
  // steps (kStepDoubles each; entry values and reciprocal pivots transcribed
  // after every refactorisation: lblk[tr_dst] = lu[tr_src], lblk[trd_dst] =
  // 1/lu[trd_src]) and the K / G_u^T record streams (kBatchDoubles per
  // batch; block ends per lane; destinations of the K entries, rt terms and
  // G_u entries); H position of each w row, control at each G position.
  double* lblk;
  double* hscr;           // per column tile: nw x W doubles of H before it replaces P
  int tr_n, trd_n;
  const int *tr_dst, *tr_src, *trd_dst, *trd_src;
  double *kstr, *gstr;
  int kst_nbat, kb_n, gst_nbat, gt_nb;
  const int *kb_end, *gt_end, *kdst, *krt_dst, *gdst, *hpos, *grow;
  // per column tile: the L-sweep steps that can change its panel (entries of
  // 4 ints as DevSweep::meta, then the idle step); null = every step
  const int *lsk_ptr, *lsk_meta;
  const int *lsk_gptr[2], *lsk_gmeta[2];   // the same, grouped as DevSweep::gmeta
  // wave-resident refactorisation (rw_ok): task records, per-lane data
  int rw_ok, rw_nnz_u, rw_nlev, rw_ntask, rw_lane_pad;
  const int *rw_wbeg, *rw_levend, *rw_rec, *rw_lane, *rw_ustart;
  int rw_split, rw_split_grid;
  // staged refactorisation of a large network: one launch per level over
  // rf_level_grid work-groups (the most any level needs) instead of one
  // work-group walking every level
  int rf_per_level, rf_level_grid;      // levels 1..rw_split: one launch per level, a task per WG
  const int* rw_lanelu;             // per task step and lane: LU position of the U entry, or -1
  const int* rf_lmeta;    // 6 ints per refactorisation level
  int rf_lds_doubles;
  const double* k_cdiag;
  // evaluation gather
  int d_total, d_lu, d_gu, d_a, d_g, d_h, src_u, src_total;
  const int *eg_ptr, *eg_idx;
  const double *eg_coef, *eg_cst;
  // workspaces
  double* src;        // [LF | u | pd | qd]
  double* dst;        // [luval | gu | a | g | h]
  double* hl;         // 10 per line
  double* kval;       // nnz_k
  double* rt;         // nw: condensed residual rt in w order
  double* pw;         // nw: step in w order (recovery)
  double* vtmp;       // nu: scratch vector (Cholesky solve)
  double* rinv;       // nx: reciprocal pivots written by the refactorisation
  const int* rf_info; // per refactorisation slot: row, lu_ptr, lu_ptr+1, diag, op0, nops
  double* panel;      // global panel workspace (when not in LDS)
  double* zcols;      // nx x (nu+1), column-major: Z = S e_j per column, then d (internal x order)
  double* psicols;    // nx x (nu+1): Psi = G_x^{-T} H_x per column, then that of the RHS column
  double* rpart;      // 2 x kRecChunks x nx partial sums of the recovery
  size_t panel_doubles;
  int* status;        // [0] Cholesky status, [1] failing index, [2] small pivot flag, [3] pivot row
  long long* trace;   // in-kernel phase timestamps of work-group 0 (null = off)
};

// Per-instance arguments of a batched launch (device array, one per
// instance; pointers to device memory).
struct BatchArg {
  const double *x, *u, *lam, *y, *sig_x, *sig_u, *sig_s, *r;
  double* K;
  long ldk;
  double* rhs;            // condensation: output; solve: input
  double* p;              // solve: the step (packed p_u p_x p_s p_lambda p_y)
  double delta;           // solve: delta_w
  double *sig_s_keep, *bwork, *cinv, *lrow;   // the handle's own buffers
  int* status;
  int nu, m;
};
// One condensation launch of a batch: the members of one panel width and
// placement, their column tiles contiguous in the tile table from tile0.
struct CondClass {
  int width = 1, nw = 1, tile0 = 0, ntiles = 0;
  bool lds = true, meta_global = false;
  size_t lds_bytes = 0;
};
// Host-side shape of a batch: maxima over the instances for the grids and
// dynamic LDS of the batched launches.
struct BatchShape {
  int count = 0;
  bool any_wave = false, any_staged = false;
  std::vector<CondClass> cls;   // condensation launches
  int max_split = 0, max_split_grid = 0;   // refactorisation levels run one launch each
  int max_staged_levels = 0, max_staged_grid = 0;
  int max_lines = 0, max_dst = 0, max_nnz_k = 0, max_nw = 0, max_nx = 0, max_nu = 0, max_m = 0;
  size_t lds_wave = 0, lds_staged = 0;
  std::vector<int> orders;   // order (nu) of each instance's condensed matrix
};
// Condensation of every instance (eval, K assembly, rt, refactorisation,
// columns with the right-hand side, symmetrisation) and the solve with
// recovery from the stored columns (Cholesky, backward substitution, p_x,
// p_lambda, p_s, p_y); nets, args, tiles are device arrays.
hipError_t launch_batch_condense(const DevNet* nets, const BatchArg* args, const int2* tiles,
                                 const BatchShape& sh, hipStream_t st);
hipError_t launch_batch_solve(const DevNet* nets, const BatchArg* args, const BatchShape& sh,
                              hipStream_t st);
struct IpmDev;
// Evaluation of a lockstep batch of interior-point solvers (rh_ipm_batch_step):
// derivative values at args' (x, u, lam, y) with the Hessian (trial = 0) or
// without it at the trial points (trial = 1, args hold wt), and the objective
// of each active instance into its f[trial].
hipError_t launch_batch_ipm_eval(const DevNet* nets, const BatchArg* args, const IpmDev* ipms,
                                 const double* sc, const BatchShape& sh, int trial,
                                 hipStream_t st);
// out[5 b + i] = status word i of instance b (device array of 5 count ints)
hipError_t launch_batch_status(const DevNet* nets, int count, int* out, hipStream_t st);

hipError_t launch_eval(const DevNet& d, const double* x, const double* u, const double* lam,
                       const double* y, bool hessian, hipStream_t st);
// sig_s_keep (optional): receives a copy of sig_s.
hipError_t launch_assemble_k(const DevNet& d, const double* sig_x, const double* sig_u,
                             const double* sig_s, double* sig_s_keep, hipStream_t st);
hipError_t launch_refactor(const DevNet& d, hipStream_t st);
hipError_t launch_rtilde(const DevNet& d, const double* r, const double* sig_s, hipStream_t st);
// mode 0: identity columns [col0, col0 + ncols) (col == nu: the right-hand-side column)
hipError_t launch_condense(const DevNet& d, int col0, int ncols, int width, bool lds,
                           const double* r, double* K, long ldk, double* rhs, hipStream_t st);
// recovery of p_x and p_lambda from p_u (one column; the handle's panel
// width and placement, whose records the sweeps read)
hipError_t launch_recover(const DevNet& d, int width, bool lds, const double* pu,
                          const double* r, double* p, hipStream_t st);
// x = scale * G_x^{-1} b (or G_x^{-T} b) [+ x if accumulate] with the factors
// of the last refactorisation (b, x natural order; one wave).
hipError_t launch_gx_solve(const DevNet& d, int width, bool lds, bool transpose, const double* b,
                           double* x, double scale, bool accumulate, hipStream_t st);
// Recovery from the stored columns of the last condensation (which included
// the right-hand-side column): p_x = Z p_u + d, p_lambda = -(Psi p_u + Psi_rhs).
hipError_t launch_recover_stored(const DevNet& d, double* p, hipStream_t st);
// hstat (optional, pinned host int[5]): receives the status words.
hipError_t launch_finish_step(const DevNet& d, const double* r, const double* sig_s, double* p,
                              int* hstat, hipStream_t st);
// K = (K + K^T) / 2 in place; copy (optional, same leading dimension): the result again.
hipError_t launch_symmetrize(double* K, long ldk, int n, double* copy, hipStream_t st);
// Cholesky of the lower triangle of K + delta I in place (K holds L on
// return), the forward substitution L y = b_in folded into the factorisation
// (b_in is read by the first launch only and may be b; y is written to b,
// which then also holds partial sums) and the backward substitution
// L^T x = y into x. status[0..1] (device, set by the first launch): 0, or 1
// and the first column whose pivot is not positive. Workspaces: dl (chol_inv_doubles(n)), X (chol_lrow_doubles(n):
// the inverses of the diagonal super-blocks of L^T). trace (optional,
// device int64[192]): wall-clock stamps of the diagonal work-group of the
// first 24 factorisation launches (8 k + 0: start, + 1: panel k - 1 applied,
// + 2: slice factored, + 3: stores issued).
hipError_t launch_cholesky_solve(double* K, long ldk, int n, double delta, const double* b_in,
                                 double* b, double* x, double* dl, double* X, int* status,
                                 hipStream_t st, long long* trace = nullptr);
// The same for every instance of a batch (orders[i] = order of instance i;
// args[i]: K, ldk, delta, bwork (b), p (x), cinv (dl), lrow (X), status).
hipError_t launch_batch_cholesky(const BatchArg* args, const std::vector<int>& orders,
                                 hipStream_t st);
// Panel columns per super-block of an order with nbk 32-column panels: one
// super-block up to 24 panels (order 768), 16 panels (512 columns) above.
__host__ __device__ constexpr int chol_superblock(int nbk) { return nbk <= 24 ? nbk : 16; }
// The same with no workspace argument: the workspaces live in a static device
// array of the library (one per device, shared by every call on it), for
// orders up to kNoallocMaxOrder; b is copied there first and left unchanged.
// hipErrorInvalidValue past the maximum order.
constexpr int kNoallocMaxOrder = 1024;
hipError_t launch_cholesky_solve_noalloc(double* K, long ldk, int n, double delta, const double* b,
                                         double* x, int* status, hipStream_t st);
// Kernel launches of one launch_cholesky_solve (status clear excluded).
int chol_launches(int n);
// Doubles of the Cholesky workspaces of order n (dl and X above).
constexpr size_t chol_inv_doubles(int n) { return 2 * size_t((n + 31) / 32) * 32 * 32; }
constexpr size_t chol_lrow_doubles(int n) {
  return size_t((n + 31) / 32) * 32 * size_t((n + 31) / 32) * 32;
}
hipError_t launch_eval_objective(const DevNet& d, const double* u, double* f, hipStream_t st);
int max_lds_bytes();
int device_cus();   // compute units of the current device
// LDS one row of the refactorisation stages (row, U sources, pivots, schedule).
size_t refactor_lds_per_row(const DevNet& d);
// Dynamic LDS of one condensation work-group: the staged step metadata and
// stream block ends, after the panels P and H (2 nw + 1 rows of `width`
// doubles) when those live in LDS.
// Dynamic LDS of a condensation work-group of `waves` waves (1 or
// kCondWaves; several only for one column with the panel in LDS).
size_t condense_lds_bytes(const DevNet& d, int width, bool lds_panels, int waves);
// Allow the LDS-staged kernels dynamic LDS up to the device's maximum.
void prepare_lds_kernels();

}  // namespace rh
