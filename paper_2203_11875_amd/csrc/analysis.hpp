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

constexpr int kKRowBlock = 256;
constexpr int kMaxRowBlocks = 16;   // LDS-resident panels: nu + nx <= 16 * 256
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

// Per-line record written by the line-evaluation kernel (doubles).
enum LineSlot : int {
  LF_PF = 0, LF_QF = 1, LF_PT = 2, LF_QT = 3,
  LF_DPF = 4, LF_DQF = 8, LF_DPT = 12, LF_DQT = 16,   // 4 partials each
  LF_SF2 = 20, LF_ST2 = 21, LF_DSF2 = 22, LF_DST2 = 26,
  LF_STRIDE = 32
};
// Local variable order of a line: theta_from, theta_to, Vm_from, Vm_to.
// Symmetric 4x4 blocks are stored as 10 entries (upper triangle, row major).
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
  std::vector<int> lev_lanes; // lanes that cooperate on one row in each level
  // Padded per-level layout: level l holds rows lev_ptr[l] .. lev_ptr[l+1]
  // (R of them) and lev_len[l] entry columns; entry k of the r-th row sits at
  // lev_base[l] + k * R + r, so its address needs no row pointer. Padding
  // entries point at their own row with source -1 (value 0).
  std::vector<int> lev_base, lev_len;
  std::vector<int> ell_col, ell_src;
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
  // K rows in blocks of kKRowBlock (one row per thread of the condensation
  // work-group), padded to the longest row of the block: entry k of row
  // kKRowBlock*b + t sits at kb_base[b] + k*kKRowBlock + t; kell_pos maps
  // each slot to its CSR entry (-1 = padding, value 0, column = own row).
  std::vector<int> kb_base, kb_len, kell_col, kell_pos;
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

// Host refactorisation + sweeps (for CPU tests of the schedule).
rh_status host_solve(const Symbolic& sym, const double* gx_values_natural_csr,
                     const double* b_nat, double* z_nat, bool transpose);
rh_status check_levels(const Symbolic& sym);

}  // namespace rh
