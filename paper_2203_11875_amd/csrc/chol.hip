// Dense FP64 Cholesky of the condensed matrix and the solve K_cond p_u = b
// (Section 3.3: the condensed KKT system is factorised by a dense Cholesky
// every iteration; Section 4.3 times it in the "Chol." column of Table 3).
//
// Blocked right-looking factorisation of the lower triangle of A + delta I
// with 32-column panels, one launch per panel k:
//  * panel work-groups, one per 32-row block i >= k, apply the rank-32 update
//    of panel k - 1 to the diagonal tile (k, k) and to their own tile on
//    MFMA, then factor the 64 x 32 slice [A_kk; A_ik] in LDS: every one of
//    them yields L_kk (redundantly) and its own L_ik = A_ik L_kk^{-T};
//  * trailing work-groups apply the panels before k to the tiles right of
//    column k: to the next column every launch, to the others four panels at
//    a time (a rank-128 update every fourth launch);
//  * the forward substitution L y = b rides along (b_i -= L_{i,k-1} y_{k-1}
//    in the panel work-groups, y_k = L_kk^{-1} b_k), y written over b;
//  * identity rows: the columns are grouped in super-blocks of S = 32 SB
//    (SB panels; SB = all panels for orders up to 768). Beside every
//    super-block the factorisation carries the rows of the S x S identity
//    (row block r joins at its own panel), which it turns into
//    I L_SS^{-T} = L_SS^{-T}: exact zeros below the diagonal, the inverse of
//    each diagonal super-block of L^T at a cost of S^2 n / 3 flops in all.
// The backward substitution L^T x = y is then one upper-triangular
// matrix-vector product per super-block, x_S = L_SS^{-T} y_S, and between two
// of them one product y_c -= L_{S,c}^T x_S over the columns left of S: one
// launch for orders up to 768, 2 ceil(n / 512) - 1 launches above.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <vector>

#include "device.hpp"

namespace rh {

namespace {

constexpr int CB = 32;          // panel width
constexpr int kTraceLaunches = 24;   // launches stamped when a trace buffer is given
constexpr int kThreads = 256;   // four waves per work-group

typedef double d4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

__device__ __forceinline__ double lane_read(double v, int lane) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_readlane(int(b & 0xffffffffll), lane);
  const int hi = __builtin_amdgcn_readlane(int(b >> 32), lane);
  return __builtin_bit_cast(double, (long long)(((unsigned long long)(unsigned)hi << 32) |
                                                (unsigned long long)(unsigned)lo));
}

// p[i] when ok, else 0. The load is unconditional (no load in a divergent
// branch); a lane that is not ok reads *safe, an address that is always
// valid (the matrix origin), never p itself, which may point past the
// matrix for a quadrant beyond its last row or column.
__device__ __forceinline__ double ld0(const double* p, size_t i, bool ok, const double* safe) {
  const double v = *(ok ? p + i : safe);
  return ok ? v : 0.0;
}

// One instance: A (lower triangle, column-major, leading dimension ld) is
// factored in place; b_in holds the right-hand side (read by launch 0 only,
// which writes every row of it, updated, to b); b receives y = L^{-1} b_in
// and then the backward substitution's partial sums; x receives the
// solution. dl: nbk 32 x 32 tiles; X: the inverse super-blocks.
struct Inst {
  double* A;
  long ld;
  int n;
  double delta;
  const double* b_in;
  double* b;
  double* x;
  double* dl;
  double* X;
  int* status;
};

struct Geo {
  int nbk, sb, S, nsb;
};
__device__ __forceinline__ Geo geo(int n) {
  Geo g;
  g.nbk = (n + CB - 1) / CB;
  g.sb = chol_superblock(g.nbk);
  g.S = g.sb * CB;
  g.nsb = (g.nbk + g.sb - 1) / g.sb;
  return g;
}

// 16 x 16 quadrant of a 32 x 32 tile in the accumulator layout of
// v_mfma_f64_16x16x4f64 computing the transposed product: lane li + 16 kk,
// register e holds element (row li, column 4 e + kk) of the quadrant whose
// (0, 0) element is base[0] (column-major, leading dimension ld); rows at or
// past rows_ok and columns at or past cols_ok read as zero.
__device__ __forceinline__ d4_t quad_load(const double* base, long ld, int rows_ok, int cols_ok,
                                          int li, int kk, const double* safe) {
  d4_t v;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = 4 * e + kk;
    v[e] = ld0(base, (size_t)c * ld + li, li < rows_ok && c < cols_ok, safe);
  }
  return v;
}
__device__ __forceinline__ void quad_store(double* base, long ld, int rows_ok, int cols_ok, int li,
                                           int kk, d4_t v, bool lower_only, int roff, int coff) {
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int c = 4 * e + kk;
    if (li < rows_ok && c < cols_ok && (!lower_only || c + coff <= li + roff))
      base[(size_t)c * ld + li] = v[e];
  }
}

// acc -= Lr Lc^T over the 32 columns of a panel: lr points at the panel's
// rows of the output quadrant (lr[q ld + li] = Lr(li, q)), lc at its
// columns; rows of lr at or past r_ok and of lc at or past c_ok are zero.
__device__ __forceinline__ d4_t quad_update(d4_t acc, const double* lr, long ldr, int r_ok,
                                            const double* lc, long ldc, int c_ok, int li, int kk,
                                            const double* safe) {
  double av[CB / 4], bv[CB / 4];
#pragma unroll
  for (int s = 0; s < CB / 4; ++s) {
    const int q = 4 * s + kk;
    av[s] = -ld0(lc, (size_t)q * ldc + li, li < c_ok, safe);
    bv[s] = ld0(lr, (size_t)q * ldr + li, li < r_ok, safe);
  }
#pragma unroll
  for (int s = 0; s < CB / 4; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s], bv[s], acc, 0, 0, 0);
  return acc;
}

// ---------------------------------------------------------------- panel
// 1 / x to the last bit or so: the hardware reciprocal refined by two Newton
// steps (x a positive normal number here; other values are flagged by the
// caller as non-positive pivots).
__device__ __forceinline__ double rcp_nr(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}

// In-place factorisation of the 64 x 32 slice P (LDS): rows 0..31 hold the
// symmetric diagonal tile D (both triangles), rows 32..63 a tile B. On
// return rows 0..31 hold L = chol(D) (zero above the diagonal) and rows
// 32..63 hold B L^{-T}. Wave w owns columns 8 w .. 8 w + 7 (lane = row, one
// register per column). Column block s (eight columns) is eliminated by its
// wave alone in registers: pivot j reads row j of the block from lane j
// (the working matrix is symmetric, so row j's entries right of the pivot
// are column j's entries below it) and updates every row's later columns,
//   T_ic <- alpha_j T_ic - 2^-e_j T_ij T_jc   (d_j = T_jj = alpha_j 2^e_j),
// which is 2^-e_j d_j times the usual Schur update: no division or square
// root sits on the pivot-to-pivot chain. Column j of L is T_.j / sqrt(sigma_j
// d_j) (sigma_j: the product of the alphas before pivot j). The block's
// columns go through LDS as they are, T (zero above the diagonal), with the
// weights 1 / (sigma_j d_j): the waves to its right apply the rank-8 update
// sum_j T_ij T_cj / (sigma_j d_j) = sum_j L_ij L_cj to their own columns,
// while the eliminating wave scales its columns to L off that chain.
// Returns the first column whose pivot is not positive, or -1.
constexpr int PS = CB + 1;   // LDS row stride of the slice
__device__ __forceinline__ int panel_factor(double (*P)[PS], double (*Lx)[8][64],
                                            double (*Lw)[8], int wave, int lane) {
  double a[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) a[t] = P[lane][8 * wave + t];
  int fl = -1;
  double sd[8];   // sigma_j d_j of the wave's own pivots
  for (int s = 0; s < 4; ++s) {
    double (*lb)[64] = Lx[s & 1];
    double* lw = Lw[s & 1];
    if (wave == s) {
      double sigma = 1.0;
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const int j = 8 * s + jj;
        const double d = lane_read(a[jj], j);
        int e;
        const double alpha = frexp(d, &e);
        sd[jj] = sigma * d;
        sigma *= alpha;
        const double bi = ldexp(-a[jj], -e);
#pragma unroll
        for (int cc = jj + 1; cc < 8; ++cc) a[cc] = fma(bi, lane_read(a[cc], j), alpha * a[cc]);
      }
      // publish T (zero above the diagonal) and the weights
#pragma unroll
      for (int jj = 0; jj < 8; ++jj) {
        const int j = 8 * s + jj;
        a[jj] = lane < j ? 0.0 : a[jj];
        lb[jj][lane] = a[jj];
      }
      if (lane < 8) {
        double v = sd[0];
#pragma unroll
        for (int jj = 1; jj < 8; ++jj) v = lane == jj ? sd[jj] : v;
        lw[lane] = rcp_nr(v);
      }
    }
    if (s < 3) lds_sync();
    if (wave == s) {
      // scale the own columns to L while the next wave updates its columns
#pragma unroll
      for (int jj = 7; jj >= 0; --jj) {
        if (!(sd[jj] > 0.0)) fl = 8 * s + jj;
        a[jj] *= rsqrt(sd[jj]);
      }
    } else if (wave > s) {
      double lr[8];
#pragma unroll
      for (int m = 0; m < 8; ++m) lr[m] = lb[m][lane] * lw[m];
#pragma unroll
      for (int t = 0; t < 8; ++t) {
        const int c = 8 * wave + t;
#pragma unroll
        for (int m = 0; m < 8; ++m) a[t] = fma(-lr[m], lb[m][c], a[t]);
      }
    }
  }
#pragma unroll
  for (int t = 0; t < 8; ++t) P[lane][8 * wave + t] = a[t];
  return fl;
}

enum { ROLE_DIAG = 0, ROLE_ROWS = 1, ROLE_IDENT = 2 };

// A panel work-group of launch k (see the file comment). ROLE_DIAG: the
// diagonal tile with the identity tile (kap, kap) below it, which yields
// L_kk^{-T}; it also writes y_k and the delayed factor tile. ROLE_ROWS: row
// block bi = k + idx. ROLE_IDENT: identity row block r = idx < kap of the
// super-block, whose tile (r, kap) holds the contributions of the panels
// before k - 1 (none when r = kap - 1).
__device__ __forceinline__ void chol_panel(const Inst& c, const Geo& G, int k, int role, int idx,
                                           long long* trace) {
  __shared__ double P[2 * CB][PS];
  __shared__ double Lx[2][8][64];
  __shared__ double Lw[2][8];
  __shared__ double red[CB], bks[CB];
  __shared__ int fails[4];
  const int n = c.n;
  const long ld = c.ld;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, kk = lane >> 4, qi = wave >> 1, qj = wave & 1;
  const int k0 = k * CB, pc0 = k0 - CB;
  const int sg = k / G.sb, kap = k - sg * G.sb, s0 = sg * G.sb;
  double* Xs = c.X + (size_t)sg * G.S * G.S;
  const bool tr = trace != nullptr && role == ROLE_DIAG && tid == 0 && k < kTraceLaunches;
  if (tr) trace[8 * k] = wall_clock64();
  // launch 0 skips the status test and its diagonal group, the only writer
  // of the status in a launch, clears it first
  if (k == 0 && role == ROLE_DIAG && tid == 0) {
    c.status[0] = 0;
    c.status[1] = 0;
  }
  const int bsz = min(CB, n - k0);
  const int bi = k + idx;   // ROLE_ROWS
  // own tile: (0, 0) element, leading dimension, valid rows; and its rows of
  // panel k - 1
  const double* own = nullptr;
  const double* opan = nullptr;
  long lo = ld;
  int orows = 0;
  bool own_load = false;
  if (role == ROLE_ROWS) {
    own = c.A + (size_t)k0 * ld + bi * CB;
    opan = c.A + (size_t)pc0 * ld + bi * CB;
    orows = n - bi * CB;
    own_load = true;
  } else if (role == ROLE_IDENT) {
    lo = G.S;
    own = Xs + (size_t)(kap * CB) * G.S + idx * CB;
    opan = Xs + (size_t)((kap - 1) * CB) * G.S + idx * CB;
    orows = CB;
    own_load = idx < kap - 1;   // tile (kap - 1, kap) gets its first contribution now
  }
  const bool dq = !(qi == 0 && qj == 1);   // the strictly upper quadrant of D is mirrored
  double bval = 0.0;
  if (role != ROLE_IDENT && tid < CB) {
    const int row = (role == ROLE_DIAG ? k0 : bi * CB) + tid;
    if (row < n) bval = (k == 0 ? c.b_in : c.b)[row];
  }
  // the factor tile of launch k - 1 (stored to A by this launch's diagonal
  // group), requested now so that its latency is not at the tail
  double dlv[CB * CB / kThreads];
#pragma unroll
  for (int j = 0; j < CB * CB / kThreads; ++j)
    dlv[j] = (role == ROLE_DIAG && k > 0) ? c.dl[(size_t)(k - 1) * CB * CB + tid + j * kThreads] : 0.0;
  const double* dbase = c.A + (size_t)(k0 + qj * 16) * ld + k0 + qi * 16;
  const double* safe = c.A;
  d4_t dacc = quad_load(dbase, ld, dq ? n - k0 - qi * 16 : 0, n - k0 - qj * 16, li, kk, safe);
  if (k == 0 && dq) {
#pragma unroll
    for (int e = 0; e < 4; ++e)
      if (qi == qj && li == 4 * e + kk && k0 + qi * 16 + li < n) dacc[e] += c.delta;
  }
  d4_t oacc = own_load ? quad_load(own + (size_t)(qj * 16) * lo + qi * 16, lo,
                                   orows - qi * 16, bsz - qj * 16, li, kk, safe)
                       : d4_t{0.0, 0.0, 0.0, 0.0};
  double bpart = 0.0;
  if (k > 0) {
    // panel k - 1: L(k, k-1) for the diagonal tile, the own rows for the own tile
    const double* lk = c.A + (size_t)pc0 * ld + k0;
    dacc = quad_update(dacc, lk + qi * 16, ld, dq ? n - k0 - qi * 16 : 0, lk + qj * 16, ld,
                       n - k0 - qj * 16, li, kk, safe);
    if (role != ROLE_DIAG)
      oacc = quad_update(oacc, opan + qi * 16, lo, orows - qi * 16, lk + qj * 16, ld,
                         n - k0 - qj * 16, li, kk, safe);
    if (role != ROLE_IDENT && qj == 0) {
      // b_rows -= L(rows, k-1) y_{k-1} (y_{k-1} was written over b)
      const double* lr = role == ROLE_DIAG ? lk : opan;
      const int rok = role == ROLE_DIAG ? n - k0 : orows;
#pragma unroll
      for (int s = 0; s < CB / 4; ++s) {
        const int q = 4 * s + kk;
        bpart = fma(ld0(lr, (size_t)q * ld + qi * 16 + li, qi * 16 + li < rok, safe), c.b[pc0 + q],
                    bpart);
      }
      bpart += __shfl_xor(bpart, 16);
      bpart += __shfl_xor(bpart, 32);
    }
  }
  if (tr) {
    asm volatile("" ::"v"(dacc[0]));
    trace[8 * k + 1] = wall_clock64();
  }
  if (qj == 0 && kk == 0) red[qi * 16 + li] = bpart;
  // D goes to both triangles of the slice from its lower triangle (the
  // elimination reads rows right of the pivot; A's upper triangle of a
  // diagonal tile is not kept up to date)
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int rl = qi * 16 + li, cl = qj * 16 + 4 * e + kk;
    if (dq && cl <= rl) {
      const double v = (rl >= bsz || cl >= bsz) ? (rl == cl ? 1.0 : 0.0) : dacc[e];
      P[rl][cl] = v;
      P[cl][rl] = v;
    }
    P[CB + rl][cl] = role == ROLE_DIAG ? (rl == cl ? 1.0 : 0.0) : oacc[e];
  }
  lds_sync();
  if (tid < CB) bks[tid] = bval - red[tid];
  const int fl = panel_factor(P, Lx, Lw, wave, lane);
  if (lane == 0) fails[wave] = fl;
  __syncthreads();
  if (tr) trace[8 * k + 2] = wall_clock64();
  int first = -1;
#pragma unroll
  for (int w = 0; w < 4; ++w)
    if (fails[w] >= 0 && (first < 0 || fails[w] < first)) first = fails[w];
  if (first >= 0 && first < bsz) {
    if (role == ROLE_DIAG && tid == 0) {
      c.status[1] = k0 + first;
      c.status[0] = 1;
    }
    return;
  }
  if (role == ROLE_ROWS) {
    for (int e = tid; e < CB * CB; e += kThreads) {
      const int r = e % CB, col = e / CB;
      if (bi * CB + r < n && col < bsz) c.A[(size_t)(k0 + col) * ld + bi * CB + r] = P[CB + r][col];
    }
    if (tid < CB && bi * CB + tid < n) c.b[bi * CB + tid] = bks[tid];
    return;
  }
  if (role == ROLE_IDENT) {
    for (int e = tid; e < CB * CB; e += kThreads) {
      const int r = e % CB, col = e / CB;
      Xs[(size_t)(kap * CB + col) * G.S + idx * CB + r] = P[CB + r][col];
    }
    return;
  }
  // ROLE_DIAG
  const bool last = k + 1 == G.nbk;
#pragma unroll
  for (int j = 0; j < CB * CB / kThreads; ++j) {
    const int e = tid + j * kThreads;
    const int r = e % CB, col = e / CB;
    Xs[(size_t)(kap * CB + col) * G.S + kap * CB + r] = P[CB + r][col];   // L_kk^{-T}
    if (last) {
      if (col <= r && k0 + r < n) c.A[(size_t)(k0 + col) * ld + k0 + r] = P[r][col];
    } else {
      c.dl[(size_t)k * CB * CB + e] = P[r][col];
    }
    // tile (k - 1, k - 1) is read by no work-group of this launch
    if (k > 0 && col <= r) c.A[(size_t)(pc0 + col) * ld + pc0 + r] = dlv[j];
  }
  if (tid < bsz) {   // y_k = L_kk^{-1} b_k, over b_k
    double v = 0.0;
#pragma unroll 8
    for (int s = 0; s < CB; ++s) v = fma(P[CB + s][tid], bks[s], v);
    c.b[k0 + tid] = v;
  }
  if (tr) trace[8 * k + 3] = wall_clock64();
}

// Trailing update of launch k >= 1 with the panels pf .. k - 1 not yet
// applied, pf = G floor((k - 1) / G) (G = kGroup): when k is a multiple of G,
// every tile right of column k (rank 32 G: work-group t covers the 2 x 2
// tiles bi = k + 1 + 2 RI + (w >> 1), bj = k + 1 + 2 RJ + (w & 1), RJ <= RI,
// regions enumerated row by row); otherwise only column k + 1, the next
// panel's (work-group t covers bi = k + 1 + 4 t + w). A tile then has every
// panel before its own column's but the last applied when its column comes
// up, and is read and written once per G launches instead of every launch.
// One 32 x 32 tile per wave, A_ij -= sum_p L(bi, p) L(bj, p)^T on MFMA.
constexpr int kGroup = 4;
__device__ __forceinline__ void chol_trailing(const Inst& c, int k, int t) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, kk = lane >> 4;
  const int nbk = (c.n + CB - 1) / CB;
  int bi, bj;
  if (k % kGroup == 0) {
    int ri = 0;
    while (t > ri) {
      t -= ri + 1;
      ++ri;
    }
    bi = k + 1 + 2 * ri + (wave >> 1);
    bj = k + 1 + 2 * t + (wave & 1);
  } else {
    bi = k + 1 + 4 * t + wave;
    bj = k + 1;
  }
  if (bi >= nbk || bj > bi) return;
  const int n = c.n;
  const long ld = c.ld;
  const int r0 = bi * CB, c0 = bj * CB;
  const bool diag = bi == bj;
  d4_t acc[2][2];
#pragma unroll
  for (int qi = 0; qi < 2; ++qi)
#pragma unroll
    for (int qj = 0; qj < 2; ++qj) {
      double* base = c.A + (size_t)(c0 + qj * 16) * ld + r0 + qi * 16;
      acc[qi][qj] = (diag && qi < qj) ? d4_t{0.0, 0.0, 0.0, 0.0}
                                      : quad_load(base, ld, n - r0 - qi * 16, n - c0 - qj * 16,
                                                  li, kk, c.A);
    }
  for (int p = kGroup * ((k - 1) / kGroup); p < k; ++p) {
    const double* lr = c.A + (size_t)p * CB * ld + r0;
    const double* lc = c.A + (size_t)p * CB * ld + c0;
    double bv[2][CB / 4], av[2][CB / 4];
#pragma unroll
    for (int q = 0; q < 2; ++q) {
#pragma unroll
      for (int s = 0; s < CB / 4; ++s) {
        const int col = 4 * s + kk;
        bv[q][s] = ld0(lr, (size_t)col * ld + q * 16 + li, r0 + q * 16 + li < n, c.A);
        av[q][s] = -ld0(lc, (size_t)col * ld + q * 16 + li, c0 + q * 16 + li < n, c.A);
      }
    }
#pragma unroll
    for (int s = 0; s < CB / 4; ++s)
#pragma unroll
      for (int qi = 0; qi < 2; ++qi)
#pragma unroll
        for (int qj = 0; qj < 2; ++qj)
          if (!(diag && qi < qj))
            acc[qi][qj] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[qj][s], bv[qi][s],
                                                               acc[qi][qj], 0, 0, 0);
  }
#pragma unroll
  for (int qi = 0; qi < 2; ++qi)
#pragma unroll
    for (int qj = 0; qj < 2; ++qj)
      if (!(diag && qi < qj))
        quad_store(c.A + (size_t)(c0 + qj * 16) * ld + r0 + qi * 16, ld, n - r0 - qi * 16,
                   n - c0 - qj * 16, li, kk, acc[qi][qj], diag, qi * 16, qj * 16);
}

// Work-groups of the trailing update of launch k (see chol_trailing).
__host__ __device__ __forceinline__ int chol_trailing_groups(int nbk, int k) {
  const int T = nbk - 1 - k;
  if (k < 1 || T < 1) return 0;
  if (k % kGroup == 0) {
    const int R = (T + 1) / 2;
    return R * (R + 1) / 2;
  }
  return (T + 3) / 4;
}

// Identity tile (r, cc) of the super-block, r < kap < cc:
// X(r, cc) -= X(r, kap-1) L(s0 + cc, k-1)^T (the first contribution, r =
// kap - 1, starts from zero).
__device__ __forceinline__ void chol_ident_trailing(const Inst& c, const Geo& G, int k, int r,
                                                    int cc) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, kk = lane >> 4, qi = wave >> 1, qj = wave & 1;
  const int sg = k / G.sb, kap = k - sg * G.sb, s0 = sg * G.sb;
  const int n = c.n;
  const long ld = c.ld;
  double* Xs = c.X + (size_t)sg * G.S * G.S;
  double* base = Xs + (size_t)(cc * CB + qj * 16) * G.S + r * CB + qi * 16;
  const int cg = (s0 + cc) * CB + qj * 16, pc0 = (k - 1) * CB;
  d4_t acc = r < kap - 1 ? quad_load(base, G.S, CB, CB, li, kk, c.A) : d4_t{0.0, 0.0, 0.0, 0.0};
  acc = quad_update(acc, Xs + (size_t)((kap - 1) * CB) * G.S + r * CB + qi * 16, G.S, CB,
                    c.A + (size_t)pc0 * ld + cg, ld, n - cg, li, kk, c.A);
  quad_store(base, G.S, CB, CB, li, kk, acc, false, 0, 0);
}

// Work-group bid of launch k: [diag | rows | identity panels | identity
// trailing | trailing regions | delta].
__device__ __forceinline__ void chol_step(const Inst& c, int k, int bid, long long* trace) {
  if (k > 0 && c.status[0] != 0) return;
  const Geo G = geo(c.n);
  if (k >= G.nbk) return;
  const int sg = k / G.sb, kap = k - sg * G.sb, sbn = min(G.sb, G.nbk - sg * G.sb);
  const int nA = G.nbk - k, nB = kap, nDc = sbn - 1 - kap;
  const int nD = kap >= 1 ? kap * nDc : 0;
  const int nC = chol_trailing_groups(G.nbk, k);
  int t = bid;
  if (t < nA) {
    chol_panel(c, G, k, t == 0 ? ROLE_DIAG : ROLE_ROWS, t, trace);
    return;
  }
  t -= nA;
  if (t < nB) {
    chol_panel(c, G, k, ROLE_IDENT, t, trace);
    return;
  }
  t -= nB;
  if (t < nD) {
    chol_ident_trailing(c, G, k, t / nDc, kap + 1 + t % nDc);
    return;
  }
  t -= nD;
  if (t < nC) {
    chol_trailing(c, k, t);
    return;
  }
  t -= nC;
  if (t == 0 && k == 0) {   // delta on the diagonal past the first tile (first tile: in registers)
    for (int i = CB + threadIdx.x; i < c.n; i += kThreads) c.A[(size_t)i * c.ld + i] += c.delta;
  }
}

// Work-groups of launch k for an order-n factorisation.
__host__ __device__ __forceinline__ int chol_step_groups(int n, int k) {
  const int nbk = (n + CB - 1) / CB;
  if (n <= 0 || k >= nbk) return 0;
  const int sb = chol_superblock(nbk);
  const int sg = k / sb, kap = k - sg * sb;
  const int sbn = sb < nbk - sg * sb ? sb : nbk - sg * sb;
  return (nbk - k) + kap + (kap >= 1 ? kap * (sbn - 1 - kap) : 0) + chol_trailing_groups(nbk, k) +
         (k == 0 ? 1 : 0);
}

// ------------------------------------------------ backward substitution
// Step t of the backward pass (super-blocks from the last): t even:
// x_S = L_SS^{-T} y_S for super-block S = nsb - 1 - t / 2 (16 rows per
// work-group, 16 column slices per row summed through LDS); t odd:
// y_c -= L_{S,c}^T x_S for the columns c left of S (32 per work-group, a
// wave per 8 columns, lanes over the rows of S).
constexpr int kBxRows = 16;

__device__ __forceinline__ void chol_back(const Inst& c, int t, int bid) {
  if (c.status[0] != 0) return;
  const Geo G = geo(c.n);
  const int sgi = G.nsb - 1 - t / 2;
  if (sgi < 0) return;
  const int n = c.n, tid = threadIdx.x;
  const int r0 = sgi * G.S, r1 = min(r0 + G.S, n);
  if ((t & 1) == 0) {
    __shared__ double part[kThreads];
    const int i0 = r0 + bid * kBxRows;
    if (i0 >= r1) return;
    const double* Xs = c.X + (size_t)sgi * G.S * G.S;
    const int li = tid % kBxRows, pj = tid / kBxRows, np = kThreads / kBxRows;
    const int row = i0 + li;
    const int jb = (i0 / CB) * CB;   // tiles left of the row's block are not stored
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int j = jb + pj;
    for (; j + 3 * np < r1; j += 4 * np) {
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int jj = j + u * np;
        acc[u] = fma(Xs[(size_t)(jj - r0) * G.S + (row - r0)], c.b[jj], acc[u]);
      }
    }
    for (; j < r1; j += np) acc[0] = fma(Xs[(size_t)(j - r0) * G.S + (row - r0)], c.b[j], acc[0]);
    part[tid] = (acc[0] + acc[1]) + (acc[2] + acc[3]);
    __syncthreads();
    if (tid < kBxRows && row < r1) {
      double v = 0.0;
      for (int p = 0; p < np; ++p) v += part[p * kBxRows + tid];
      c.x[row] = v;
    }
    return;
  }
  if (sgi == 0) return;
  const int c0 = bid * CB;
  if (c0 >= r0) return;
  const int wave = tid >> 6, lane = tid & 63;
  constexpr int kMaxRowsPerLane = 12;   // S <= 768
  double xv[kMaxRowsPerLane];
#pragma unroll
  for (int m = 0; m < kMaxRowsPerLane; ++m) {
    const int i = r0 + lane + 64 * m;
    xv[m] = i < r1 ? c.x[i] : 0.0;
  }
  for (int q = 0; q < 8; ++q) {
    const int col = c0 + 8 * wave + q;
    const double* Lc = c.A + (size_t)col * c.ld;
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < kMaxRowsPerLane; ++m) {
      const int i = r0 + lane + 64 * m;
      s = fma(ld0(Lc, i, i < r1, c.A), xv[m], s);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o);
    if (lane == 0) c.b[col] -= s;
  }
}

// Work-groups of backward step t, and the number of backward steps.
__host__ __device__ __forceinline__ int chol_back_groups(int n, int t) {
  if (n <= 0) return 0;
  const int nbk = (n + CB - 1) / CB;
  const int sb = chol_superblock(nbk), S = sb * CB, nsb = (nbk + sb - 1) / sb;
  const int sgi = nsb - 1 - t / 2;
  if (sgi < 0) return 0;
  if ((t & 1) == 0) {
    const int rows = S < n - sgi * S ? S : n - sgi * S;
    return (rows + kBxRows - 1) / kBxRows;
  }
  return sgi == 0 ? 0 : sgi * sb;
}
__host__ __device__ __forceinline__ int chol_back_steps(int n) {
  if (n <= 0) return 0;
  const int nbk = (n + CB - 1) / CB;
  const int sb = chol_superblock(nbk);
  return 2 * ((nbk + sb - 1) / sb) - 1;
}

__global__ void __launch_bounds__(kThreads) k_chol(Inst c, int k, long long* trace) {
  chol_step(c, k, blockIdx.x, trace);
}
__global__ void __launch_bounds__(kThreads) k_chol_back(Inst c, int t) {
  chol_back(c, t, blockIdx.x);
}
__global__ void k_chol_clear(int* status) {
  if (threadIdx.x < 2) status[threadIdx.x] = 0;
}

__device__ __forceinline__ Inst batch_inst(const BatchArg& q) {
  return Inst{q.K, q.ldk, q.nu, q.delta, q.bwork, q.bwork, q.p, q.cinv, q.lrow, q.status};
}
__global__ void __launch_bounds__(kThreads) k_chol_b(const BatchArg* __restrict__ a, int k) {
  const Inst c = batch_inst(cst(a, blockIdx.z));
  if ((int)blockIdx.x >= chol_step_groups(c.n, k)) return;
  chol_step(c, k, blockIdx.x, nullptr);
}
__global__ void __launch_bounds__(kThreads) k_chol_back_b(const BatchArg* __restrict__ a, int t) {
  const Inst c = batch_inst(cst(a, blockIdx.z));
  if ((int)blockIdx.x >= chol_back_groups(c.n, t)) return;
  chol_back(c, t, blockIdx.x);
}

}  // namespace

int chol_launches(int n) {
  if (n <= 0) return 0;
  return (n + CB - 1) / CB + chol_back_steps(n);
}

hipError_t launch_cholesky_solve(double* K, long ldk, int n, double delta, const double* b_in,
                                 double* b, double* x, double* dl, double* X, int* status,
                                 hipStream_t st, long long* trace) {
  if (n <= 0) {
    hipLaunchKernelGGL(k_chol_clear, dim3(1), dim3(64), 0, st, status);
    return hipGetLastError();
  }
  const Inst c{K, ldk, n, delta, b_in, b, x, dl, X, status};
  const int nbk = (n + CB - 1) / CB;
  for (int k = 0; k < nbk; ++k)
    hipLaunchKernelGGL(k_chol, dim3(chol_step_groups(n, k)), dim3(kThreads), 0, st, c, k, trace);
  const int nb = chol_back_steps(n);
  for (int t = 0; t < nb; ++t) {
    const int g = chol_back_groups(n, t);
    if (g > 0) hipLaunchKernelGGL(k_chol_back, dim3(g), dim3(kThreads), 0, st, c, t);
  }
  return hipGetLastError();
}

hipError_t launch_batch_cholesky(const BatchArg* args, const std::vector<int>& orders, hipStream_t st) {
  const int B = (int)orders.size();
  if (B == 0) return hipSuccess;
  int max_nbk = 0, max_back = 0;
  for (int n : orders) {
    max_nbk = std::max(max_nbk, (n + CB - 1) / CB);
    max_back = std::max(max_back, chol_back_steps(n));
  }
  for (int k = 0; k < max_nbk; ++k) {
    int grid = 0;
    for (int n : orders) grid = std::max(grid, chol_step_groups(n, k));
    if (grid > 0) hipLaunchKernelGGL(k_chol_b, dim3(grid, 1, B), dim3(kThreads), 0, st, args, k);
  }
  for (int t = 0; t < max_back; ++t) {
    int grid = 0;
    for (int n : orders) grid = std::max(grid, chol_back_groups(n, t));
    if (grid > 0) hipLaunchKernelGGL(k_chol_back_b, dim3(grid, 1, B), dim3(kThreads), 0, st, args, t);
  }
  return hipGetLastError();
}

// ------------------------------------------------ allocation-free solve
// Workspace of launch_cholesky_solve_noalloc: every device the library runs
// on holds one copy until the process ends. Layout (doubles): the
// right-hand-side work vector (kNoallocMaxOrder), the diagonal factor tiles
// (chol_inv_doubles), then the inverse super-blocks (the largest over
// orders <= kNoallocMaxOrder: 768^2 at a single 24-panel super-block).
namespace {
constexpr size_t kNoallocX = 768 * 768;
constexpr size_t kNoallocDoubles =
    size_t(kNoallocMaxOrder) + chol_inv_doubles(kNoallocMaxOrder) + kNoallocX;
static __device__ __align__(256) double scratch[kNoallocDoubles];

std::mutex g_scratch_mu;
double* g_scratch_ptr[64] = {};   // device address of `scratch` per device ordinal

size_t x_doubles(int n) {
  const int nbk = (n + CB - 1) / CB, sb = chol_superblock(nbk);
  return size_t((nbk + sb - 1) / sb) * size_t(sb * CB) * size_t(sb * CB);
}
}  // namespace

hipError_t noalloc_scratch(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

hipError_t launch_cholesky_solve_noalloc(double* K, long ldk, int n, double delta, const double* b,
                                         double* x, int* status, hipStream_t st) {
  if (n < 0 || n > kNoallocMaxOrder || x_doubles(n) > kNoallocX) return hipErrorInvalidValue;
  double* base = nullptr;
  const hipError_t e = noalloc_scratch(&base);
  if (e != hipSuccess) return e;
  double* bw = base;
  double* dl = bw + kNoallocMaxOrder;
  double* X = dl + chol_inv_doubles(kNoallocMaxOrder);
  return launch_cholesky_solve(K, ldk, n, delta, b, bw, x, dl, X, status, st, nullptr);
}

}  // namespace rh
