// One-time host symbolic analysis of a power network for the condensation
// hot path: index maps, fixed sparsity patterns, fill-reducing symmetric
// ordering of G_x, symbolic LU with static diagonal pivots, level sets of the
// four triangular sweeps, the refactorisation schedule and the gather lists
// the evaluation kernels follow. Plain C++ (no HIP), so it runs and is tested
// on a machine without a GPU.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "rhipm.h"

namespace rh {

constexpr int kKRowBlock = 64;      // rows per block of the row-blocked record layouts
constexpr int kRefLdsBudget = 155 * 1024;   // bytes of LDS the refactorisation may use
// Wave-resident refactorisation: 8 waves; a task is one row of at most 64
// LU entries (one lane per entry) or up to four rows of at most 16 entries
// (one 16-lane row each). Per task: a record of kRwRec ints
// {lane-data offset, steps, wide, 0, rp0[4], len[4], nlow[4], ustart[4],
// row[4]} (per row of the task: first LU position, entries, lower entries,
// first LDS slot of its U entries, row index) and, per lane, the packed
// 16-bit U indices of its steps (two steps per int, ceil(steps / 2) ints).
constexpr int kRwWaves = 8;
constexpr int kRwRec = 24;
constexpr int kRwPacked = 32;
// a level is factored by the multi-work-group kernel while some wave of the
// single work-group would run at least this many tasks in it
constexpr int kRwSplitMin = 3;
// Condensation sweep steps: entries a lane holds in registers, most lanes
// per row (one DPP row), threads of the work-group, ints of step metadata.
constexpr int kSweepPF = 8;
constexpr int kSweepMaxLanes = 64;
constexpr int kSweepThreads = 64;
constexpr int kSweepMeta = 4;
// Waves of a condensation work-group with one column and LDS panels: the
// steps of one level are spread over them, and the record streams split.
// Two counts: kCondWaves and kCondWavesWide (grouped lists for each are
// built; index 0 and 1 of the per-count arrays).
constexpr int kCondWaves = 4;
constexpr int kCondWavesWide = 8;
// two waves: the record streams split, every sweep on one wave
constexpr int kCondWavesPair = 2;
inline int wave_index(int nw) { return nw == kCondWavesWide ? 1 : 0; }
// Row-blocked record streams of the condensation (K, G_u^T): batches of
// kStreamBatch records per lane.
constexpr int kStreamBatch = 8;
// Device record sizes in doubles: a sweep lane block (kSweepPF values,
// kSweepPF 32-bit offsets, pivot, row offset + pad) and a stream batch.
// Device record layouts (doubles). A sweep step: 7 chunks of 64 lanes x 16
// bytes (values 0-1, 2-3, 4-5, 6-7; offsets 0-3, 4-7; reciprocal pivot, row
// offset, writer flag), so that each 16-byte load of the wave is contiguous.
// A stream batch: 6 such chunks (values 0-1 .. 6-7; offsets 0-3, 4-7).
constexpr int kChunk = 2 * kSweepThreads;           // doubles per chunk
constexpr int kStepDoubles = 7 * kChunk;
constexpr int kBatchDoubles = 6 * kChunk;

// Per-line record written by the line-evaluation kernel: LF_STRIDE slots of
// nl doubles each, slot k of line l at k nl + l (consecutive lines, i.e.
// consecutive threads, write consecutive doubles).
enum LineSlot : int {
  LF_PF = 0, LF_QF = 1, LF_PT = 2, LF_QT = 3,
  LF_DPF = 4, LF_DQF = 8, LF_DPT = 12, LF_DQT = 16,   // 4 partials each
  LF_SF2 = 20, LF_ST2 = 21, LF_DSF2 = 22, LF_DST2 = 26,
  LF_STRIDE = 32
};
// Local variable order of a line: theta_from, theta_to, Vm_from, Vm_to.
// Symmetric 4x4 blocks are stored as 10 entries (upper triangle, row major),
// entry k of line l at k nl + l.
constexpr int HL_STRIDE = 10;
inline int hl_index(int a, int b) {   // a <= b
  static const int base[4] = {0, 4, 7, 9};
  return base[a] + (b - a);
}

// A triangular sweep in level order. Row lists and entries are stored level
// by level so that one level is a contiguous range.
struct Sweep {
  int nlev = 0;
  std::vector<int> lev_ptr;   // nlev + 1 offsets into rows
  std::vector<int> rows;      // row (internal index) per slot
  std::vector<int> ptr;       // slot -> entry range (size n + 1)
  std::vector<int> col;       // entry -> column (internal index)
  std::vector<int> src;       // entry -> position in the LU value array
  bool has_diag = false;      // divide by the diagonal (U-type sweeps)
  std::vector<int> diag_src;  // slot -> position of the diagonal in LU values
  // Schedule of the condensation kernel's sweeps, in steps of one wave. A
  // step holds R rows with S = 2^ls lanes per row (S <= kSweepMaxLanes),
  // TL = R * S lanes in use; lane t = r * S + k takes entries k + j * S
  // (j < kSweepPF) of its row r. A step owns TL + 1 lane blocks (the last,
  // all padding, serves the idle lanes); per block: kSweepPF (column, LU
  // position) pairs (position -1 = padding), the row, whether this lane
  // writes the row (the last lane of its group) and the LU position of the
  // pivot (U-type sweeps, writing lanes). Rows with nothing to do (no entries
  // in a unit-diagonal sweep) are left out.
  int ks_nstep = 0;
  std::vector<int> ks_meta;        // kSweepMeta ints per step: first block, TL, ls, 0
  int lb_n = 0;                    // lane blocks
  std::vector<int> lb_col, lb_src; // kSweepPF per block
  std::vector<int> lb_row, lb_wr, lb_dsrc;   // per block (row 0, wr 0 on padding blocks)
};

struct Gather {          // dst[e] = c[e] + sum_t coef[t] * src[idx[t]]
  std::vector<int> ptr;
  std::vector<int> idx;
  std::vector<double> coef;
  std::vector<double> cst;
};

struct KGather {         // K assembly lists
  std::vector<int> hl_ptr, hl_idx;           // W part: HL entries
  std::vector<int> ata_ptr, ata_a1, ata_a2, ata_row;   // A^T Sigma A part
  std::vector<int> diag_var;                 // entry -> w variable if diagonal, else -1
};

struct Symbolic {
  // sizes
  int nb = 0, nl = 0, ng = 0, nx = 0, nu = 0, m = 0, nw = 0, nlim = 0;
  int ref = -1, ref_gen = -1;
  double base = 100.0;
  // host copy of the data the kernels need
  std::vector<double> pd, qd;
  std::vector<int> lf, lt;               // line ends
  std::vector<double> gff, bff, gft, bft;   // pi-model admittances per line
  std::vector<double> c2, c1;
  // natural index maps
  std::vector<int> th_nat, vmx_nat, vmu;   // per bus (-1 if absent)
  std::vector<int> pg_u;                   // per generator (-1 for reference)
  std::vector<int> gen_of_bus;             // per bus (-1 if none)
  std::vector<int> lim_of_line;            // per line: limited-line ordinal or -1
  std::vector<int> x_kind, x_bus, u_kind, u_ref;
  std::vector<int> g_row_of_x;             // natural g row paired with natural x (identity)
  // symmetric pivot order: perm[k] = natural x index of internal k
  std::vector<int> perm, iperm;
  // per line: w index (= [u ; x internal]) of its 4 local variables, -1 if none
  std::vector<int> line_w;                 // 4 * nl
  // per line: weight sources for the Hessian kernel (natural indices, -1 = none)
  //   lamP/lamQ at each end, yQg at each end, y of flow rows
  std::vector<int> line_wsrc;              // 8 * nl
  std::vector<int> ref_lines, ref_ends;    // lines incident to the reference bus
  // LU pattern (internal), combined rows sorted, diagonal present
  std::vector<int> lu_ptr, lu_col, lu_diag;
  // natural G_x CSR pattern and map to LU positions
  std::vector<int> gx_ptr, gx_col, gx_lu;
  // refactorisation schedule (rows in L-level order)
  std::vector<int> rf_rowslot;             // L sweep slots reused
  std::vector<int> rf_kptr;                // per LU lower entry (by row order) -> op range
  std::vector<int> rf_op_src, rf_op_dst;   // U source position, destination position
  std::vector<int> rf_lower_ptr;           // per internal row: first lower-entry id
  int max_row = 0;
  int max_row_ops = 0;                     // refactorisation multiply-adds of one row
  int max_row_lower = 0;                   // lower entries of one row
  std::vector<int> rf_piv;                 // per LU position (lower entries): pivot position
  std::vector<int> rf_dst_local;           // per op: destination offset within its row
  long refactor_ops = 0;
  // sweeps
  Sweep sl, su, sut, slt;
  // G_u (rows internal, cols u) CSR and CSC; A (rows natural h, cols w) CSR and CSC
  std::vector<int> gu_ptr, gu_col, gucsc_ptr, gucsc_row, gucsc_from_csr;
  std::vector<int> a_ptr, a_col, acsc_ptr, acsc_row, acsc_from_csr;
  // K pattern (w x w), CSR with sorted columns
  std::vector<int> k_ptr, k_col;
  KGather kg;
  // Row-blocked record streams (one row per lane of the condensation's
  // wave): the rows, sorted by length (row[p] = row at stream position p,
  // -1 past the end; pos = its inverse), in blocks of kKRowBlock; position
  // p = kKRowBlock*b + t belongs to lane t; lane t's records, block after
  // block (each block padded to its longest row), form one stream of
  // nbat * kStreamBatch records, record q of lane t at t * nbat *
  // kStreamBatch + q; end[b] = records per lane through block b.
  // kind: 0 padding (value 0, column 0), 1 matrix entry (src = its position
  // in the CSR values of K / G_u),
  // 2 extra term of the row (K: rt, column nw; G_u^T: -H_u of the row, column
  // = the row). K columns are w indices; G_u^T columns internal state rows.
  struct LaneStream {
    int nbat = 0;
    std::vector<int> row, pos, end, col, src, kind;
  };
  LaneStream kst, gst;
  // refactorisation launch shape per level: lanes per row and the LDS
  // layout of one row's staging area (in doubles): stride, offsets of the U
  // sources, the pivots, the destination offsets and the op pointers
  std::vector<int> rf_lmeta;               // 6 per level
  int rf_lds_doubles = 0;                  // LDS the refactorisation needs
  // wave-resident refactorisation (used when every LU row has at most 64
  // entries and U plus the pivot reciprocals fit in LDS)
  bool rw_ok = false;
  int rw_nnz_u = 0;                        // U entries held in LDS; slot rw_nnz_u is 0
  std::vector<int> rw_wbeg;                // kRwWaves + 1: first task of each wave
  std::vector<int> rw_levend;              // kRwWaves * nlev: end of each level per wave
  std::vector<int> rw_rec;                 // kRwRec ints per task (wave-major order)
  std::vector<int> rw_lane;                // per-lane task data (see analysis.cpp)
  std::vector<int> rw_ustart;              // nx: first LDS slot of each row's U entries
  // levels 1 .. rw_split run one task per work-group, one launch per level
  // (levels with many tasks per wave); per step and lane of a task, the LU
  // position of the U entry it subtracts (-1: none), at record field 3
  int rw_split = 0;
  int rw_split_grid = 0;                   // largest task count of one wave in those levels
  std::vector<int> rw_lanelu;
  std::vector<double> k_cdiag;             // constant diagonal (2 c2 base^2 on Pg)
  std::vector<int> sig_map;                // w -> index into [Sigma_u ; Sigma_x(natural)]
  // evaluation gather: dst = [luval | gu | a | g(natural) | h]
  Gather eg;
  int d_lu = 0, d_gu = 0, d_a = 0, d_g = 0, d_h = 0, d_total = 0;
  int src_u = 0, src_total = 0;            // src = [LF | u]
  double cost_rank1 = 0.0;                 // 2 c2_ref base^2 (enters Sigma of A row 0)
  std::string error;
};

// Returns RH_OK or an error code (message in sym.error).
rh_status analyze(const rh_network_desc& d, const rh_options* opts, Symbolic& sym);

// The condensation's device records for launch width W: panel offsets are
// bytes from the start of a work-group's panels, P = [V; Z; indicator]
// (nw + 1 rows, natural order) then H (nw rows in K-stream order: H row v at
// position kst.pos[v]); W doubles per row. The output of G_u^T Psi - H_u is
// written over P's first nu rows in G-stream order (control gst.row[p] at p).
struct CondenseRecords {
  std::vector<double> steps;         // kStepDoubles per step (all sweeps, idle steps)
  std::vector<int> meta[4];          // per sweep, per step: {global step, ls, 0, 0}; then idle
  std::vector<int> tr_dst, tr_src;   // steps[tr_dst] = LU value tr_src
  std::vector<int> trd_dst, trd_src; // steps[trd_dst] = 1 / LU value trd_src
  std::vector<double> kstr, gstr;    // kBatchDoubles per batch
  std::vector<int> kdst;             // nnz_k: kstr index of each K entry (CSR)
  std::vector<int> krt_dst;          // nw: kstr index of each row's rt term
  std::vector<int> gdst;             // nnz_gu: gstr index of each G_u entry (CSR)
  std::vector<int> hpos;             // nw: H position of w row v
  std::vector<int> grow;             // nu: control at G-stream position p
  // per column tile (W identity columns, the last tile with the right-hand
  // side): the L-sweep step entries (as meta[0]) that can change its panel,
  // then the idle step; lsk_ptr in entries of 4 ints
  std::vector<int> lsk_ptr, lsk_meta;
  // the step lists for work-groups of NW waves (group_for_waves), [c] for
  // NW = kCondWaves (c = 0) and kCondWavesWide (c = 1): per sweep NW lists
  // of ngrp + 1 entries, wave after wave; per column tile the same for its
  // L-sweep steps (lsk_gptr in entries)
  std::vector<int> gmeta[2][4];
  int ngrp[2][4] = {{0, 0, 0, 0}, {0, 0, 0, 0}};
  std::vector<int> lsk_gptr[2], lsk_gmeta[2];
};
void build_condense_records(const Symbolic& sym, int W, CondenseRecords& out);
int group_for_waves(const int* entries, size_t n_with_idle, int nwaves, std::vector<int>& out);
// The number of groups group_for_waves makes of a sweep's steps.
int wave_groups(const Sweep& sw, int nwaves);

// Host refactorisation + sweeps (for CPU tests of the schedule).
rh_status host_solve(const Symbolic& sym, const double* gx_values_natural_csr,
                     const double* b_nat, double* z_nat, bool transpose);
rh_status check_levels(const Symbolic& sym);
// Host emulation of the condensation kernel on its device records for width
// W (random G_x with dominant diagonal, G_u, K, rt and r4 values drawn from
// seed), columns 0, nu/2 and the right-hand side (ncols of them), against a
// dense computation; the largest error relative to each column's largest
// entry.
rh_status host_check_condense(const Symbolic& sym, int W, uint64_t seed, int ncols,
                              double* max_rel_err);

}  // namespace rh
