// Host symbolic analysis (see analysis.hpp).
//
// The state Jacobian G_x of the polar power-flow equations has the structure
// of the network: the P balance at bus i (paired with theta_i) and the Q
// balance at a PQ bus i (paired with Vm_i) depend on theta_j and Vm_j of i and
// its neighbours. Its pattern is therefore structurally symmetric under that
// pairing, and a symmetric permutation with pivots on the diagonal keeps the
// strong diagonal of the power-flow Jacobian. The paper refactorises G_x on
// the GPU with a fixed pattern and fixed permutations computed once on the
// host (Section 3.1, SpRF; Section 4.2); this file computes that fixed data.
#include "analysis.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <complex>
#include <cstring>
#include <numeric>
#include <set>
#include <utility>

namespace rh {

namespace {

rh_status fail(Symbolic& s, rh_status st, const std::string& msg) {
  s.error = msg;
  return st;
}

int find_pos(const std::vector<int>& ptr, const std::vector<int>& col, int r, int c) {
  auto b = col.begin() + ptr[r];
  auto e = col.begin() + ptr[r + 1];
  auto it = std::lower_bound(b, e, c);
  if (it == e || *it != c) return -1;
  return int(it - col.begin());
}

void to_csr(int nrow, std::vector<std::vector<int>>& rows, std::vector<int>& ptr,
            std::vector<int>& col) {
  ptr.assign(nrow + 1, 0);
  col.clear();
  for (int r = 0; r < nrow; ++r) {
    auto& v = rows[r];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    ptr[r + 1] = ptr[r] + int(v.size());
    col.insert(col.end(), v.begin(), v.end());
  }
}

void transpose(int nrow, int ncol, const std::vector<int>& ptr, const std::vector<int>& col,
               std::vector<int>& tptr, std::vector<int>& trow, std::vector<int>& from) {
  tptr.assign(ncol + 1, 0);
  for (int c : col) tptr[c + 1]++;
  for (int c = 0; c < ncol; ++c) tptr[c + 1] += tptr[c];
  trow.assign(col.size(), 0);
  from.assign(col.size(), 0);
  std::vector<int> next(tptr.begin(), tptr.end() - 1);
  for (int r = 0; r < nrow; ++r)
    for (int p = ptr[r]; p < ptr[r + 1]; ++p) {
      int q = next[col[p]]++;
      trow[q] = r;
      from[q] = p;
    }
}

// Greedy elimination ordering on an undirected graph (elimination graph kept
// explicitly), the next node the one of least key. Plain minimum degree
// (with_level false): key = (degree, node id). With a level term: key =
// (2 degree + level, level, node id), where a node's level is one more than
// the largest level of the eliminated nodes it was a neighbour of — its level
// in the L sweep and in the refactorisation. The level term trades a little
// fill for a shorter dependency chain: on the 1354- and 9241-bus networks it
// halves the levels (43 -> 22, 96 -> 43) for 1% more LU entries. Returns the
// elimination order; higher[v] receives v's neighbours at the moment it is
// eliminated, i.e. the off-diagonal pattern of its row of U.
std::vector<int> minimum_degree(int n, std::vector<std::vector<int>> adj,
                                std::vector<std::vector<int>>& higher, bool with_level) {
  std::vector<int> lev(n, 0);
  auto key = [&](int v) {
    const int d = int(adj[v].size());
    return with_level ? std::array<int, 3>{2 * d + lev[v], lev[v], v}
                      : std::array<int, 3>{d, 0, v};
  };
  std::set<std::array<int, 3>> pq;
  for (int v = 0; v < n; ++v) pq.insert(key(v));
  std::vector<int> order;
  order.reserve(n);
  higher.assign(n, {});
  std::vector<int> merged;
  while (!pq.empty()) {
    int v = (*pq.begin())[2];
    pq.erase(pq.begin());
    order.push_back(v);
    std::vector<int> nbrs = adj[v];
    higher[v] = nbrs;
    for (int u : nbrs) {
      pq.erase(key(u));
      lev[u] = std::max(lev[u], lev[v] + 1);
      merged.clear();
      std::set_union(adj[u].begin(), adj[u].end(), nbrs.begin(), nbrs.end(),
                     std::back_inserter(merged));
      std::vector<int> out;
      out.reserve(merged.size());
      for (int w : merged)
        if (w != u && w != v) out.push_back(w);
      adj[u].swap(out);
      pq.insert(key(u));
    }
    adj[v].clear();
  }
  return order;
}

// The pattern of U for a given elimination order: higher[v] = v's neighbours
// when it is eliminated (elimination graph kept explicitly, as above).
void eliminate_in_order(int n, std::vector<std::vector<int>> adj, const std::vector<int>& order,
                        std::vector<std::vector<int>>& higher) {
  higher.assign(n, {});
  std::vector<int> merged;
  for (int v : order) {
    const std::vector<int> nbrs = adj[v];
    higher[v] = nbrs;
    for (int u : nbrs) {
      merged.clear();
      std::set_union(adj[u].begin(), adj[u].end(), nbrs.begin(), nbrs.end(),
                     std::back_inserter(merged));
      std::vector<int> out;
      out.reserve(merged.size());
      for (int w : merged)
        if (w != u && w != v) out.push_back(w);
      adj[u].swap(out);
    }
    adj[v].clear();
  }
}

// Nested dissection: a part of the graph is split by a vertex separator
// taken from the middle of a breadth-first level structure rooted at a
// pseudo-peripheral node (the end of repeated breadth-first searches), and
// trimmed to the nodes that touch the far side; both sides are ordered
// recursively, then the separator. Parts of at most kLeaf nodes are ordered
// by minimum degree on their own subgraph.
std::vector<int> nested_dissection(int n, const std::vector<std::vector<int>>& adj) {
  constexpr int kLeaf = 64;
  std::vector<int> order;
  order.reserve(n);
  std::vector<int> part(n, 0), dist(n, -1), local(n, -1);
  int next_part = 1;
  // breadth-first search inside part p from r; returns the visit order
  auto bfs = [&](int r, int p, std::vector<int>& seen) {
    seen.clear();
    seen.push_back(r);
    dist[r] = 0;
    for (size_t h = 0; h < seen.size(); ++h) {
      const int v = seen[h];
      for (int w : adj[v])
        if (part[w] == p && dist[w] < 0) {
          dist[w] = dist[v] + 1;
          seen.push_back(w);
        }
    }
  };
  std::vector<int> seen;
  // order the nodes of `nodes` (all in part p); recursion by an explicit stack
  // of {nodes, part} items, the separator appended after both sides
  struct Item {
    std::vector<int> nodes;
    int p;
    std::vector<int> sep;   // appended when the item is popped the second time
    bool done;
  };
  auto order_leaf = [&](const std::vector<int>& nodes, int p) {
    std::vector<std::vector<int>> sub(nodes.size());
    for (size_t i = 0; i < nodes.size(); ++i) local[nodes[i]] = int(i);
    for (size_t i = 0; i < nodes.size(); ++i) {
      for (int w : adj[nodes[i]])
        if (part[w] == p) sub[i].push_back(local[w]);
      std::sort(sub[i].begin(), sub[i].end());
    }
    std::vector<std::vector<int>> h;
    for (int v : minimum_degree(int(nodes.size()), sub, h, false)) order.push_back(nodes[v]);
  };
  std::vector<Item> stack;
  stack.push_back({{}, 0, {}, false});
  stack.back().nodes.resize(n);
  std::iota(stack.back().nodes.begin(), stack.back().nodes.end(), 0);
  while (!stack.empty()) {
    Item it = std::move(stack.back());
    stack.pop_back();
    if (it.done) {
      order.insert(order.end(), it.sep.begin(), it.sep.end());
      continue;
    }
    const int p = it.p;
    if (int(it.nodes.size()) <= kLeaf) {
      order_leaf(it.nodes, p);
      continue;
    }
    // connected component of the first node; other components are split off
    for (int v : it.nodes) dist[v] = -1;
    bfs(it.nodes[0], p, seen);
    if (seen.size() < it.nodes.size()) {
      const int q = next_part++;
      Item rest{{}, q, {}, false};
      for (int v : it.nodes)
        if (dist[v] < 0) {
          part[v] = q;
          rest.nodes.push_back(v);
        }
      const int q2 = next_part++;
      Item comp{{}, q2, {}, false};
      for (int v : seen) part[v] = q2;
      comp.nodes = seen;
      stack.push_back(std::move(rest));
      stack.push_back(std::move(comp));
      continue;
    }
    // pseudo-peripheral root: restart from the farthest node while the
    // eccentricity grows
    int root = seen.back(), ecc = dist[seen.back()];
    for (int rep = 0; rep < 8; ++rep) {
      for (int v : it.nodes) dist[v] = -1;
      bfs(root, p, seen);
      const int far = seen.back();
      if (dist[far] <= ecc && rep > 0) break;
      ecc = dist[far];
      root = far;
    }
    for (int v : it.nodes) dist[v] = -1;
    bfs(root, p, seen);
    // middle level: the first level at which half the nodes are reached
    const int half = int(seen.size()) / 2;
    const int mid = std::max(1, dist[seen[half]]);
    const int qa = next_part++, qb = next_part++;
    Item a{{}, qa, {}, false}, b{{}, qb, {}, false};
    std::vector<int> sep;
    for (int v : seen) {
      if (dist[v] < mid) {
        a.nodes.push_back(v);
      } else if (dist[v] > mid) {
        b.nodes.push_back(v);
      } else {
        sep.push_back(v);
      }
    }
    // a separator node with no neighbour beyond the middle level joins side a
    std::vector<int> kept;
    for (int v : sep) {
      bool touches_b = false;
      for (int w : adj[v])
        if (part[w] == p && dist[w] > mid) {
          touches_b = true;
          break;
        }
      if (touches_b)
        kept.push_back(v);
      else
        a.nodes.push_back(v);
    }
    if (b.nodes.empty() || kept.empty()) {   // no split (a star-like part)
      order_leaf(it.nodes, p);
      continue;
    }
    for (int v : a.nodes) part[v] = qa;
    for (int v : b.nodes) part[v] = qb;
    for (int v : kept) part[v] = -1;
    stack.push_back({{}, p, kept, true});
    stack.push_back(std::move(a));
    stack.push_back(std::move(b));
  }
  return order;
}

bool build_sweep(Sweep& sw, int n, const std::vector<int>& level, int nlev,
                 const std::vector<std::vector<std::pair<int, int>>>& entries,
                 bool has_diag, const std::vector<int>& diag_pos) {
  sw.nlev = nlev;
  sw.has_diag = has_diag;
  std::vector<std::vector<int>> bylev(nlev);
  for (int i = 0; i < n; ++i) bylev[level[i]].push_back(i);
  sw.lev_ptr.assign(nlev + 1, 0);
  sw.rows.clear();
  sw.ptr.assign(1, 0);
  sw.col.clear();
  sw.src.clear();
  sw.diag_src.clear();
  for (int l = 0; l < nlev; ++l) {
    for (int i : bylev[l]) {
      sw.rows.push_back(i);
      for (auto& e : entries[i]) {
        sw.col.push_back(e.first);
        sw.src.push_back(e.second);
      }
      sw.ptr.push_back(int(sw.col.size()));
      if (has_diag) sw.diag_src.push_back(diag_pos[i]);
    }
    sw.lev_ptr[l + 1] = int(sw.rows.size());
  }
  // Condensation schedule: per level, the rows with work sorted by length
  // (longest first, ties by slot), cut into steps of at most
  // kSweepThreads / S rows, S the fewest lanes (a power of two) that leave
  // each lane at most kSweepPF entries of the step's longest row.
  sw.ks_nstep = 0;
  sw.ks_meta.clear();
  sw.lb_n = 0;
  sw.lb_col.clear();
  sw.lb_src.clear();
  sw.lb_row.clear();
  sw.lb_wr.clear();
  sw.lb_dsrc.clear();
  auto add_block = [&](int row, int wr, int dsrc) {
    sw.lb_row.push_back(row);
    sw.lb_wr.push_back(wr);
    sw.lb_dsrc.push_back(dsrc);
    ++sw.lb_n;
  };
  for (int l = 0; l < nlev; ++l) {
    std::vector<int> qs;
    for (int q = sw.lev_ptr[l]; q < sw.lev_ptr[l + 1]; ++q)
      if (has_diag || sw.ptr[q + 1] > sw.ptr[q]) qs.push_back(q);
    std::stable_sort(qs.begin(), qs.end(), [&](int a, int b) {
      return sw.ptr[a + 1] - sw.ptr[a] > sw.ptr[b + 1] - sw.ptr[b];
    });
    for (size_t i = 0; i < qs.size();) {
      const int maxlen = sw.ptr[qs[i] + 1] - sw.ptr[qs[i]];
      int ls = 0;
      while ((1 << ls) < kSweepMaxLanes && (maxlen + (1 << ls) - 1) / (1 << ls) > kSweepPF) ++ls;
      const int S = 1 << ls;
      if ((maxlen + S - 1) / S > kSweepPF) return false;
      const int R = int(std::min<size_t>(qs.size() - i, size_t(kSweepThreads / S)));
      sw.ks_meta.insert(sw.ks_meta.end(), {sw.lb_n, R * S, ls, l});
      for (int t = 0; t < R * S; ++t) {
        const int q = qs[i + t / S], k = t % S;
        for (int j = 0; j < kSweepPF; ++j) {
          const int e = sw.ptr[q] + k + j * S;
          if (e < sw.ptr[q + 1]) {
            sw.lb_col.push_back(sw.col[e]);
            sw.lb_src.push_back(sw.src[e]);
          } else {
            sw.lb_col.push_back(0);
            sw.lb_src.push_back(-1);
          }
        }
        const bool wr = k == S - 1;
        add_block(sw.rows[q], wr ? 1 : 0, wr && has_diag ? sw.diag_src[q] : -1);
      }
      for (int j = 0; j < kSweepPF; ++j) {   // the idle lanes' block
        sw.lb_col.push_back(0);
        sw.lb_src.push_back(-1);
      }
      add_block(0, 0, -1);
      ++sw.ks_nstep;
      i += R;
    }
  }
  return true;
}


// Row-blocked record stream of a CSR matrix with n rows plus one extra term
// per row (see Symbolic::LaneStream): rows sorted by length (longest first,
// ties by index) so that rows of one block have similar lengths, in blocks of
// kKRowBlock, one row per lane, each block padded to its longest row.
template <class Col, class Src, class Extra>
void build_stream(Symbolic::LaneStream& ls, int n, const std::vector<int>& ptr, Col col, Src src,
                  Extra extra_col) {
  const int nblk = (n + kKRowBlock - 1) / kKRowBlock;
  ls.row.assign(size_t(nblk) * kKRowBlock, -1);
  for (int v = 0; v < n; ++v) ls.row[v] = v;
  std::stable_sort(ls.row.begin(), ls.row.begin() + n, [&](int a, int b) {
    return ptr[a + 1] - ptr[a] > ptr[b + 1] - ptr[b];
  });
  ls.pos.assign(n, 0);
  for (int p = 0; p < n; ++p) ls.pos[ls.row[p]] = p;
  ls.end.assign(nblk, 0);
  std::vector<std::vector<int>> lc(kKRowBlock), lsrc(kKRowBlock), lk(kKRowBlock);
  int acc = 0;
  for (int bk = 0; bk < nblk; ++bk) {
    int len = 0;
    for (int t = 0; t < kKRowBlock; ++t) {
      const int v = ls.row[size_t(bk) * kKRowBlock + t];
      if (v >= 0) len = std::max(len, ptr[v + 1] - ptr[v] + 1);
    }
    for (int t = 0; t < kKRowBlock; ++t) {
      const int v = ls.row[size_t(bk) * kKRowBlock + t];
      const int nv = v >= 0 ? ptr[v + 1] - ptr[v] : 0;
      for (int k = 0; k < len; ++k) {
        if (k < nv) {
          lc[t].push_back(col(ptr[v] + k));
          lsrc[t].push_back(src(ptr[v] + k));
          lk[t].push_back(1);
        } else if (k == nv && v >= 0) {
          lc[t].push_back(extra_col(v));
          lsrc[t].push_back(v);
          lk[t].push_back(2);
        } else {
          lc[t].push_back(0);
          lsrc[t].push_back(-1);
          lk[t].push_back(0);
        }
      }
    }
    acc += len;
    ls.end[bk] = acc;
  }
  ls.nbat = std::max(1, (acc + kStreamBatch - 1) / kStreamBatch);
  const size_t per = size_t(ls.nbat) * kStreamBatch;
  ls.col.assign(per * kKRowBlock, 0);
  ls.src.assign(per * kKRowBlock, -1);
  ls.kind.assign(per * kKRowBlock, 0);
  for (int t = 0; t < kKRowBlock; ++t)
    for (int p = 0; p < acc; ++p) {
      ls.col[t * per + p] = lc[t][p];
      ls.src[t * per + p] = lsrc[t][p];
      ls.kind[t * per + p] = lk[t][p];
    }
}


}  // namespace

rh_status analyze(const rh_network_desc& d, const rh_options* opts, Symbolic& s) {
  // ------------------------------------------------------------ validation
  if (d.nb < 2 || d.nl < 1 || d.ng < 1) return fail(s, RH_ERR_ARG, "need nb>=2, nl>=1, ng>=1");
  if (!d.bus_type || !d.pd || !d.qd || !d.vmin || !d.vmax || !d.from || !d.to || !d.r ||
      !d.x || !d.b || !d.rate || !d.gen_bus || !d.c2 || !d.c1 || !d.c0 || !d.pmin ||
      !d.pmax || !d.qmin || !d.qmax)
    return fail(s, RH_ERR_ARG, "null array in network description");
  if (!(d.base_mva > 0)) return fail(s, RH_ERR_ARG, "base_mva must be positive");
  const int nb = d.nb, nl = d.nl, ng = d.ng;
  s.nb = nb;
  s.nl = nl;
  s.ng = ng;
  s.base = d.base_mva;
  s.ref = -1;
  for (int i = 0; i < nb; ++i) {
    int t = d.bus_type[i];
    if (t < 1 || t > 3) return fail(s, RH_ERR_ARG, "bus_type must be 1, 2 or 3");
    if (t == 3) {
      if (s.ref >= 0) return fail(s, RH_ERR_ARG, "more than one reference bus");
      s.ref = i;
    }
  }
  if (s.ref < 0) return fail(s, RH_ERR_ARG, "no reference bus");
  s.gen_of_bus.assign(nb, -1);
  for (int g = 0; g < ng; ++g) {
    int b = d.gen_bus[g];
    if (b < 0 || b >= nb) return fail(s, RH_ERR_ARG, "gen_bus out of range");
    if (s.gen_of_bus[b] >= 0) return fail(s, RH_ERR_ARG, "two generators on one bus");
    if (d.bus_type[b] == 1) return fail(s, RH_ERR_ARG, "generator on a PQ bus");
    s.gen_of_bus[b] = g;
  }
  for (int i = 0; i < nb; ++i)
    if (d.bus_type[i] != 1 && s.gen_of_bus[i] < 0)
      return fail(s, RH_ERR_ARG, "PV/reference bus without generator");
  s.ref_gen = s.gen_of_bus[s.ref];
  std::vector<std::vector<int>> adj(nb);
  for (int l = 0; l < nl; ++l) {
    int f = d.from[l], t = d.to[l];
    if (f < 0 || f >= nb || t < 0 || t >= nb || f == t)
      return fail(s, RH_ERR_ARG, "bad line ends");
    if (!(std::abs(d.r[l]) + std::abs(d.x[l]) > 0))
      return fail(s, RH_ERR_ARG, "zero line impedance");
    adj[f].push_back(t);
    adj[t].push_back(f);
  }
  for (auto& a : adj) {
    std::sort(a.begin(), a.end());
    a.erase(std::unique(a.begin(), a.end()), a.end());
  }
  {  // connectivity from the reference bus (else G_x is singular)
    std::vector<char> seen(nb, 0);
    std::vector<int> stack{s.ref};
    seen[s.ref] = 1;
    int cnt = 1;
    while (!stack.empty()) {
      int v = stack.back();
      stack.pop_back();
      for (int w : adj[v])
        if (!seen[w]) {
          seen[w] = 1;
          ++cnt;
          stack.push_back(w);
        }
    }
    if (cnt != nb) return fail(s, RH_ERR_SINGULAR, "network not connected to the reference bus");
  }

  // ------------------------------------------------------------- host data
  s.pd.assign(d.pd, d.pd + nb);
  s.qd.assign(d.qd, d.qd + nb);
  s.lf.assign(d.from, d.from + nl);
  s.lt.assign(d.to, d.to + nl);
  s.gff.resize(nl);
  s.bff.resize(nl);
  s.gft.resize(nl);
  s.bft.resize(nl);
  for (int l = 0; l < nl; ++l) {
    std::complex<double> ys = 1.0 / std::complex<double>(d.r[l], d.x[l]);
    s.gff[l] = ys.real();
    s.bff[l] = ys.imag() + 0.5 * d.b[l];
    s.gft[l] = -ys.real();
    s.bft[l] = -ys.imag();
  }
  s.c2.assign(d.c2, d.c2 + ng);
  s.c1.assign(d.c1, d.c1 + ng);

  // ---------------------------------------------------- natural index maps
  s.th_nat.assign(nb, -1);
  s.vmx_nat.assign(nb, -1);
  s.vmu.assign(nb, -1);
  s.pg_u.assign(ng, -1);
  int k = 0;
  for (int i = 0; i < nb; ++i)
    if (i != s.ref) s.th_nat[i] = k++;
  for (int i = 0; i < nb; ++i)
    if (d.bus_type[i] == 1) s.vmx_nat[i] = k++;
  s.nx = k;
  for (int g = 0; g < ng; ++g) s.vmu[d.gen_bus[g]] = g;
  k = ng;
  for (int g = 0; g < ng; ++g)
    if (g != s.ref_gen) s.pg_u[g] = k++;
  s.nu = k;
  s.nw = s.nu + s.nx;
  const int nx = s.nx, nu = s.nu;
  s.x_kind.assign(nx, 0);
  s.x_bus.assign(nx, 0);
  for (int i = 0; i < nb; ++i) {
    if (s.th_nat[i] >= 0) { s.x_kind[s.th_nat[i]] = 0; s.x_bus[s.th_nat[i]] = i; }
    if (s.vmx_nat[i] >= 0) { s.x_kind[s.vmx_nat[i]] = 1; s.x_bus[s.vmx_nat[i]] = i; }
  }
  s.u_kind.assign(nu, 0);
  s.u_ref.assign(nu, 0);
  for (int g = 0; g < ng; ++g) {
    s.u_kind[g] = 1;
    s.u_ref[g] = d.gen_bus[g];
    if (s.pg_u[g] >= 0) { s.u_kind[s.pg_u[g]] = 2; s.u_ref[s.pg_u[g]] = g; }
  }
  s.lim_of_line.assign(nl, -1);
  s.nlim = 0;
  for (int l = 0; l < nl; ++l)
    if (d.rate[l] > 0) s.lim_of_line[l] = s.nlim++;
  s.m = 1 + ng + 2 * s.nlim;

  // ------------------------------------------------ natural G_x pattern
  // row of a bus equation = natural x index of its paired variable
  std::vector<std::vector<int>> gxrows(nx);
  auto bus_xcols = [&](int i, std::vector<int>& out) {
    auto add_bus = [&](int j) {
      if (s.th_nat[j] >= 0) out.push_back(s.th_nat[j]);
      if (s.vmx_nat[j] >= 0) out.push_back(s.vmx_nat[j]);
    };
    add_bus(i);
    for (int j : adj[i]) add_bus(j);
  };
  for (int i = 0; i < nb; ++i) {
    if (s.th_nat[i] >= 0) bus_xcols(i, gxrows[s.th_nat[i]]);
    if (s.vmx_nat[i] >= 0) bus_xcols(i, gxrows[s.vmx_nat[i]]);
  }
  to_csr(nx, gxrows, s.gx_ptr, s.gx_col);

  // ------------------------------------------------------------- ordering
  std::vector<std::vector<int>> gadj(nx);
  for (int r = 0; r < nx; ++r)
    for (int p = s.gx_ptr[r]; p < s.gx_ptr[r + 1]; ++p)
      if (s.gx_col[p] != r) gadj[r].push_back(s.gx_col[p]);
  for (auto& a : gadj) std::sort(a.begin(), a.end());
  std::vector<std::vector<int>> higher;
  const int ordering = opts ? opts->ordering : 0;
  if (ordering == 2) {
    s.perm = nested_dissection(nx, gadj);
    eliminate_in_order(nx, gadj, s.perm, higher);
  } else if (ordering == 0 || ordering == 1) {
    s.perm = minimum_degree(nx, gadj, higher, ordering == 0);
  } else {
    return fail(s, RH_ERR_ARG, "unknown ordering");
  }
  s.iperm.assign(nx, 0);
  for (int i = 0; i < nx; ++i) s.iperm[s.perm[i]] = i;

  // ---------------------------------------------------------- symbolic LU
  std::vector<std::vector<int>> urows(nx), lrows(nx);
  for (int i = 0; i < nx; ++i) {
    for (int v : higher[s.perm[i]]) urows[i].push_back(s.iperm[v]);
    std::sort(urows[i].begin(), urows[i].end());
    for (int j : urows[i]) lrows[j].push_back(i);
  }
  s.lu_ptr.assign(nx + 1, 0);
  s.lu_col.clear();
  s.lu_diag.assign(nx, 0);
  s.max_row = 0;
  for (int i = 0; i < nx; ++i) {
    std::sort(lrows[i].begin(), lrows[i].end());
    for (int c : lrows[i]) s.lu_col.push_back(c);
    s.lu_diag[i] = int(s.lu_col.size());
    s.lu_col.push_back(i);
    for (int c : urows[i]) s.lu_col.push_back(c);
    s.lu_ptr[i + 1] = int(s.lu_col.size());
    s.max_row = std::max(s.max_row, s.lu_ptr[i + 1] - s.lu_ptr[i]);
  }
  s.gx_lu.assign(s.gx_col.size(), -1);
  for (int r = 0; r < nx; ++r)
    for (int p = s.gx_ptr[r]; p < s.gx_ptr[r + 1]; ++p) {
      int pos = find_pos(s.lu_ptr, s.lu_col, s.iperm[r], s.iperm[s.gx_col[p]]);
      if (pos < 0) return fail(s, RH_ERR_ARG, "internal: G_x entry missing from LU pattern");
      s.gx_lu[p] = pos;
    }

  // ------------------------------------------------------------- levels
  std::vector<int> levL(nx, 0), levU(nx, 0);
  int nlevL = 0, nlevU = 0;
  for (int i = 0; i < nx; ++i) {
    int lv = 0;
    for (int p = s.lu_ptr[i]; p < s.lu_diag[i]; ++p) lv = std::max(lv, levL[s.lu_col[p]] + 1);
    levL[i] = lv;
    nlevL = std::max(nlevL, lv + 1);
  }
  for (int i = nx - 1; i >= 0; --i) {
    int lv = 0;
    for (int p = s.lu_diag[i] + 1; p < s.lu_ptr[i + 1]; ++p)
      lv = std::max(lv, levU[s.lu_col[p]] + 1);
    levU[i] = lv;
    nlevU = std::max(nlevU, lv + 1);
  }
  {
    std::vector<std::vector<std::pair<int, int>>> eL(nx), eU(nx), eUT(nx), eLT(nx);
    for (int i = 0; i < nx; ++i) {
      for (int p = s.lu_ptr[i]; p < s.lu_diag[i]; ++p) {
        int c = s.lu_col[p];
        eL[i].push_back({c, p});      // L(i, c), c < i
        eLT[c].push_back({i, p});     // L^T(c, i) = L(i, c), i > c
      }
      for (int p = s.lu_diag[i] + 1; p < s.lu_ptr[i + 1]; ++p) {
        int c = s.lu_col[p];
        eU[i].push_back({c, p});      // U(i, c), c > i
        eUT[c].push_back({i, p});     // U^T(c, i) = U(i, c), i < c
      }
    }
    bool ok = build_sweep(s.sl, nx, levL, nlevL, eL, false, s.lu_diag) &&
              build_sweep(s.su, nx, levU, nlevU, eU, true, s.lu_diag);
    // U^T is lower triangular with the pattern of L (symmetric structure);
    // L^T is upper triangular with the pattern of U.
    ok = ok && build_sweep(s.sut, nx, levL, nlevL, eUT, true, s.lu_diag) &&
         build_sweep(s.slt, nx, levU, nlevU, eLT, false, s.lu_diag);
    if (!ok)
      return fail(s, RH_ERR_ARG, "an LU row has more entries than one wave's sweep step holds");
  }

  // ----------------------------------------------- refactorisation schedule
  // Row-by-row Doolittle elimination (rows in any order consistent with the
  // L levels): for each lower entry (i, k) in increasing k,
  //   l_ik = a_ik / u_kk;  a_ij -= l_ik * u_kj  for every U entry (k, j).
  s.rf_kptr.assign(s.lu_col.size() + 1, 0);
  s.rf_op_src.clear();
  s.rf_op_dst.clear();
  s.refactor_ops = 0;
  for (int i = 0; i < nx; ++i) {
    for (int p = s.lu_ptr[i]; p < s.lu_ptr[i + 1]; ++p) {
      if (p < s.lu_diag[i]) {
        int kk = s.lu_col[p];
        for (int q = s.lu_diag[kk] + 1; q < s.lu_ptr[kk + 1]; ++q) {
          int dst = find_pos(s.lu_ptr, s.lu_col, i, s.lu_col[q]);
          if (dst < 0) return fail(s, RH_ERR_ARG, "internal: LU pattern not closed");
          s.rf_op_src.push_back(q);
          s.rf_op_dst.push_back(dst);
        }
      }
      s.rf_kptr[p + 1] = int(s.rf_op_src.size());
    }
  }
  s.refactor_ops = long(s.rf_op_src.size());
  s.rf_piv.assign(s.lu_col.size(), -1);
  s.rf_dst_local.assign(s.rf_op_dst.size(), 0);
  s.max_row_ops = 0;
  s.max_row_lower = 0;
  for (int i = 0; i < nx; ++i) {
    for (int p = s.lu_ptr[i]; p < s.lu_diag[i]; ++p) s.rf_piv[p] = s.lu_diag[s.lu_col[p]];
    for (int o = s.rf_kptr[s.lu_ptr[i]]; o < s.rf_kptr[s.lu_diag[i]]; ++o)
      s.rf_dst_local[o] = s.rf_op_dst[o] - s.lu_ptr[i];
    s.max_row_ops = std::max(s.max_row_ops, s.rf_kptr[s.lu_diag[i]] - s.rf_kptr[s.lu_ptr[i]]);
    s.max_row_lower = std::max(s.max_row_lower, s.lu_diag[i] - s.lu_ptr[i]);
  }
  // Per level: as many rows in flight as the LDS allows. A row stages its
  // values, the U entries its elimination reads, its pivots (doubles) and
  // the op offsets and pointers (ints) in LDS.
  s.rf_lmeta.assign(6 * s.sl.nlev, 0);
  s.rf_lds_doubles = 0;
  for (int l = 0; l < s.sl.nlev; ++l) {
    int mrow = 1, mops = 0, mlow = 0;
    for (int q = s.sl.lev_ptr[l]; q < s.sl.lev_ptr[l + 1]; ++q) {
      const int i = s.sl.rows[q];
      mrow = std::max(mrow, s.lu_ptr[i + 1] - s.lu_ptr[i]);
      mops = std::max(mops, s.rf_kptr[s.lu_diag[i]] - s.rf_kptr[s.lu_ptr[i]]);
      mlow = std::max(mlow, s.lu_diag[i] - s.lu_ptr[i]);
    }
    const int dbl = mrow + mops + mlow;
    const int ints = mops + mlow + 1;
    const int stride = dbl + (ints + 1) / 2;
    const int rows = s.sl.lev_ptr[l + 1] - s.sl.lev_ptr[l];
    int lanes = 4;
    // fewest lanes per row (most rows in flight) whose staging fits in LDS,
    // but no more groups than rows
    while (lanes < 64 && (size_t(1024 / lanes) * stride * 8 > size_t(kRefLdsBudget) ||
                          (1024 / lanes) / 2 >= rows))
      lanes *= 2;
    if (size_t(1024 / lanes) * stride * 8 > size_t(kRefLdsBudget))
      return fail(s, RH_ERR_ARG, "a row of the LU factors is too long for the refactorisation");
    int* mt = &s.rf_lmeta[6 * l];
    mt[0] = lanes;
    mt[1] = stride;
    mt[2] = mrow;                 // offset of the U sources
    mt[3] = mrow + mops;          // offset of the pivots
    mt[4] = dbl;                  // offset (in doubles) of the int area: dst offsets
    mt[5] = mops;                 // op pointers follow the dst offsets (in ints)
    s.rf_lds_doubles = std::max(s.rf_lds_doubles, (1024 / lanes) * stride);
  }

  // --------------------------------- wave-resident refactorisation tasks
  // Each task runs on one wave. Lane (segment g, position p) holds entry p of
  // its row; at step q the multiplier of the q-th lower entry is broadcast
  // from lane q of the segment and every lane applies a_p -= l_q u_(k_q, col p)
  // with u read from LDS at its packed 16-bit index (the zero slot where the
  // row of U has no such entry). The record and the lane data are described
  // with kRwRec.
  {
    s.rw_ok = false;
    s.rw_wbeg.clear();
    s.rw_levend.clear();
    s.rw_rec.clear();
    s.rw_lane.clear();
    s.rw_lanelu.clear();
    s.rw_split = 0;
    s.rw_split_grid = 0;
    std::vector<int> ustart(nx + 1, 0);
    for (int i = 0; i < nx; ++i) ustart[i + 1] = ustart[i] + (s.lu_ptr[i + 1] - s.lu_diag[i] - 1);
    s.rw_nnz_u = ustart[nx];
    s.rw_ustart.assign(ustart.begin(), ustart.end() - 1);
    const size_t lds = (size_t(s.rw_nnz_u) + 1 + nx) * sizeof(double) +
                       size_t(kRwWaves) * s.sl.nlev * sizeof(int);
    bool ok = s.max_row <= 64 && s.rw_nnz_u < 65535 && lds <= size_t(kRefLdsBudget) &&
              !(opts && opts->refactor == 1);
    if (ok) {
      const int zslot = s.rw_nnz_u;
      struct Task { int wide; int nsteps; std::vector<int> rows; };
      std::vector<std::vector<std::vector<int>>> wave_tasks(kRwWaves);   // [wave][level] -> task ids
      std::vector<Task> tasks;
      const int nlev = s.sl.nlev;
      for (int w = 0; w < kRwWaves; ++w) wave_tasks[w].assign(nlev, {});
      // level 0 (rows without lower entries: U row and pivot are the values
      // themselves) is copied by all threads at kernel start, not in tasks
      for (int l = 1; l < nlev; ++l) {
        std::vector<int> shortr, longr;
        for (int q = s.sl.lev_ptr[l]; q < s.sl.lev_ptr[l + 1]; ++q) {
          const int i = s.sl.rows[q];
          (s.lu_ptr[i + 1] - s.lu_ptr[i] <= 16 ? shortr : longr).push_back(i);
        }
        auto nlow = [&](int i) { return s.lu_diag[i] - s.lu_ptr[i]; };
        std::stable_sort(shortr.begin(), shortr.end(),
                         [&](int a, int b) { return nlow(a) > nlow(b); });
        std::vector<int> ids;
        for (size_t g = 0; g < shortr.size(); g += 4) {
          Task t{0, 0, {}};
          for (size_t h = g; h < std::min(shortr.size(), g + 4); ++h) {
            t.rows.push_back(shortr[h]);
            t.nsteps = std::max(t.nsteps, nlow(shortr[h]));
          }
          ids.push_back(int(tasks.size()));
          tasks.push_back(t);
        }
        for (int i : longr) {
          ids.push_back(int(tasks.size()));
          tasks.push_back(Task{1, nlow(i), {i}});
        }
        // longest first to the least loaded wave
        std::stable_sort(ids.begin(), ids.end(),
                         [&](int a, int b) { return tasks[a].nsteps > tasks[b].nsteps; });
        std::vector<long> load(kRwWaves, 0);
        for (int id : ids) {
          int w = int(std::min_element(load.begin(), load.end()) - load.begin());
          load[w] += tasks[id].nsteps + 4;
          wave_tasks[w][l].push_back(id);
        }
      }
      s.rw_wbeg.assign(kRwWaves + 1, 0);
      s.rw_levend.assign(size_t(kRwWaves) * nlev, 0);
      for (int w = 0; w < kRwWaves; ++w) {
        int cnt = 0;
        for (int l = 0; l < nlev; ++l) {
          for (int id : wave_tasks[w][l]) {
            const Task& t = tasks[id];
            const int off = int(s.rw_lane.size());
            const int npk = (t.nsteps + 1) / 2;
            std::vector<int> blk(size_t(npk) * 64, int(unsigned(zslot) | (unsigned(zslot) << 16)));
            std::vector<int> lublk(size_t(t.nsteps) * 64, -1);
            int rec[kRwRec] = {off, t.nsteps, t.wide, int(s.rw_lanelu.size())};
            for (size_t g = 0; g < t.rows.size(); ++g) {
              const int i = t.rows[g], rp0 = s.lu_ptr[i], len = s.lu_ptr[i + 1] - rp0;
              const int nl = s.lu_diag[i] - rp0;
              rec[4 + g] = rp0;
              rec[8 + g] = len;
              rec[12 + g] = nl;
              rec[16 + g] = ustart[i];
              rec[20 + g] = i;
              const int lane0 = t.wide ? 0 : 16 * int(g);
              for (int q = 0; q < nl; ++q) {
                const int kr = s.lu_col[rp0 + q];
                for (int o = s.rf_kptr[rp0 + q]; o < s.rf_kptr[rp0 + q + 1]; ++o) {
                  const int p = s.rf_op_dst[o] - rp0;
                  const int u = ustart[kr] + (s.rf_op_src[o] - s.lu_diag[kr] - 1);
                  int& w2 = blk[size_t(q / 2) * 64 + lane0 + p];
                  unsigned wv = unsigned(w2);
                  if (q & 1) wv = (wv & 0xffffu) | (unsigned(u) << 16);
                  else wv = (wv & 0xffff0000u) | unsigned(u);
                  w2 = int(wv);
                  lublk[size_t(q) * 64 + lane0 + p] = s.rf_op_src[o];
                }
              }
            }
            s.rw_lane.insert(s.rw_lane.end(), blk.begin(), blk.end());
            s.rw_lanelu.insert(s.rw_lanelu.end(), lublk.begin(), lublk.end());
            s.rw_rec.insert(s.rw_rec.end(), rec, rec + kRwRec);
            ++cnt;
          }
          s.rw_levend[size_t(w) * nlev + l] = cnt;
        }
        s.rw_wbeg[w + 1] = s.rw_wbeg[w] + cnt;
      }
      // leading levels where some wave has many tasks go to the
      // multi-work-group kernel
      for (int l = 1; l < nlev; ++l) {
        int mx = 0;
        for (int w = 0; w < kRwWaves; ++w) mx = std::max(mx, int(wave_tasks[w][l].size()));
        if (mx < kRwSplitMin) break;
        s.rw_split = l;
        s.rw_split_grid = std::max(s.rw_split_grid, mx);
      }
      // a dummy record (loaded, never run, by waves past their last task)
      // pointing at one block of 64 ints that also stands in for the packed
      // steps a task does not have
      const int pad = int(s.rw_lane.size());
      int dummy[kRwRec] = {pad, 0, 0, 0};
      s.rw_rec.insert(s.rw_rec.end(), dummy, dummy + kRwRec);
      s.rw_lane.insert(s.rw_lane.end(), 64, int(unsigned(zslot) | (unsigned(zslot) << 16)));
      s.rw_ok = true;
    }
  }

  // -------------------------------------------------- w = [u ; x internal]
  auto w_theta = [&](int i) { return s.th_nat[i] >= 0 ? nu + s.iperm[s.th_nat[i]] : -1; };
  auto w_vm = [&](int i) {
    if (s.vmx_nat[i] >= 0) return nu + s.iperm[s.vmx_nat[i]];
    return s.vmu[i];
  };
  s.line_w.assign(4 * nl, -1);
  s.line_wsrc.assign(8 * nl, -1);
  for (int l = 0; l < nl; ++l) {
    int f = d.from[l], t = d.to[l];
    s.line_w[4 * l + 0] = w_theta(f);
    s.line_w[4 * l + 1] = w_theta(t);
    s.line_w[4 * l + 2] = w_vm(f);
    s.line_w[4 * l + 3] = w_vm(t);
    int* ws = &s.line_wsrc[8 * l];
    ws[0] = s.th_nat[f];                       // lambda of P balance at from (natural g row)
    ws[1] = s.vmx_nat[f];                      // lambda of Q balance at from
    ws[2] = s.th_nat[t];
    ws[3] = s.vmx_nat[t];
    ws[4] = s.gen_of_bus[f] >= 0 ? 1 + s.gen_of_bus[f] : -1;   // y of Qg
    ws[5] = s.gen_of_bus[t] >= 0 ? 1 + s.gen_of_bus[t] : -1;
    int kl = s.lim_of_line[l];
    ws[6] = kl >= 0 ? 1 + ng + kl : -1;        // y of |S_from|^2
    ws[7] = kl >= 0 ? 1 + ng + s.nlim + kl : -1;
    if (f == s.ref || t == s.ref) {
      s.ref_lines.push_back(l);
      s.ref_ends.push_back(f == s.ref ? 0 : 1);
    }
  }
  s.sig_map.assign(s.nw, 0);
  for (int v = 0; v < nu; ++v) s.sig_map[v] = v;
  for (int i = 0; i < nx; ++i) s.sig_map[nu + i] = nu + s.perm[i];

  // ---------------------------------------------------------- G_u and A
  // line-ends incident to each bus, in line order
  std::vector<std::vector<std::pair<int, int>>> ends(nb);
  for (int l = 0; l < nl; ++l) {
    ends[d.from[l]].push_back({l, 0});
    ends[d.to[l]].push_back({l, 1});
  }
  std::vector<std::vector<int>> gurows(nx), arows(s.m);
  auto bus_wcols = [&](int i, std::vector<int>& out) {
    auto add = [&](int j) {
      if (w_theta(j) >= 0) out.push_back(w_theta(j));
      out.push_back(w_vm(j));
    };
    add(i);
    for (int j : adj[i]) add(j);
  };
  auto gu_of_bus = [&](int i, int row_internal) {
    std::vector<int> wc;
    bus_wcols(i, wc);
    for (int w : wc)
      if (w < nu) gurows[row_internal].push_back(w);
  };
  for (int i = 0; i < nb; ++i) {
    if (s.th_nat[i] >= 0) {
      int ri = s.iperm[s.th_nat[i]];
      gu_of_bus(i, ri);
      int g = s.gen_of_bus[i];
      if (g >= 0 && s.pg_u[g] >= 0) gurows[ri].push_back(s.pg_u[g]);
    }
    if (s.vmx_nat[i] >= 0) gu_of_bus(i, s.iperm[s.vmx_nat[i]]);
  }
  to_csr(nx, gurows, s.gu_ptr, s.gu_col);
  transpose(nx, nu, s.gu_ptr, s.gu_col, s.gucsc_ptr, s.gucsc_row, s.gucsc_from_csr);
  bus_wcols(s.ref, arows[0]);
  for (int g = 0; g < ng; ++g) bus_wcols(d.gen_bus[g], arows[1 + g]);
  for (int l = 0; l < nl; ++l) {
    int kl = s.lim_of_line[l];
    if (kl < 0) continue;
    for (int kk = 0; kk < 4; ++kk) {
      int w = s.line_w[4 * l + kk];
      if (w >= 0) {
        arows[1 + ng + kl].push_back(w);
        arows[1 + ng + s.nlim + kl].push_back(w);
      }
    }
  }
  to_csr(s.m, arows, s.a_ptr, s.a_col);
  transpose(s.m, s.nw, s.a_ptr, s.a_col, s.acsc_ptr, s.acsc_row, s.acsc_from_csr);

  // -------------------------------------------------------------- K pattern
  std::vector<std::vector<int>> krows(s.nw);
  for (int v = 0; v < s.nw; ++v) krows[v].push_back(v);
  for (int l = 0; l < nl; ++l)
    for (int a = 0; a < 4; ++a)
      for (int b = 0; b < 4; ++b) {
        int wa = s.line_w[4 * l + a], wb = s.line_w[4 * l + b];
        if (wa >= 0 && wb >= 0) krows[wa].push_back(wb);
      }
  for (int j = 0; j < s.m; ++j)
    for (int p = s.a_ptr[j]; p < s.a_ptr[j + 1]; ++p)
      for (int q = s.a_ptr[j]; q < s.a_ptr[j + 1]; ++q) krows[s.a_col[p]].push_back(s.a_col[q]);
  to_csr(s.nw, krows, s.k_ptr, s.k_col);
  const int nnzk = int(s.k_col.size());
  {
    std::vector<std::vector<int>> hl(nnzk);
    std::vector<std::vector<std::array<int, 3>>> at(nnzk);
    for (int l = 0; l < nl; ++l)
      for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) {
          int wa = s.line_w[4 * l + a], wb = s.line_w[4 * l + b];
          if (wa < 0 || wb < 0) continue;
          int e = find_pos(s.k_ptr, s.k_col, wa, wb);
          hl[e].push_back(hl_index(std::min(a, b), std::max(a, b)) * nl + l);
        }
    for (int j = 0; j < s.m; ++j)
      for (int p = s.a_ptr[j]; p < s.a_ptr[j + 1]; ++p)
        for (int q = s.a_ptr[j]; q < s.a_ptr[j + 1]; ++q) {
          int e = find_pos(s.k_ptr, s.k_col, s.a_col[p], s.a_col[q]);
          at[e].push_back({p, q, j});
        }
    auto& kg = s.kg;
    kg.hl_ptr.assign(nnzk + 1, 0);
    kg.ata_ptr.assign(nnzk + 1, 0);
    kg.diag_var.assign(nnzk, -1);
    for (int e = 0; e < nnzk; ++e) {
      for (int v : hl[e]) kg.hl_idx.push_back(v);
      kg.hl_ptr[e + 1] = int(kg.hl_idx.size());
      for (auto& t : at[e]) {
        kg.ata_a1.push_back(t[0]);
        kg.ata_a2.push_back(t[1]);
        kg.ata_row.push_back(t[2]);
      }
      kg.ata_ptr[e + 1] = int(kg.ata_a1.size());
    }
    for (int v = 0; v < s.nw; ++v) kg.diag_var[find_pos(s.k_ptr, s.k_col, v, v)] = v;
  }
  build_stream(s.kst, s.nw, s.k_ptr, [&](int e) { return s.k_col[e]; }, [](int e) { return e; },
               [&](int) { return s.nw; });
  build_stream(s.gst, s.nu, s.gucsc_ptr, [&](int e) { return s.gucsc_row[e]; },
               [&](int e) { return s.gucsc_from_csr[e]; }, [](int q) { return q; });
  s.k_cdiag.assign(s.nw, 0.0);
  for (int g = 0; g < ng; ++g)
    if (s.pg_u[g] >= 0) s.k_cdiag[s.pg_u[g]] = 2.0 * d.c2[g] * s.base * s.base;
  s.cost_rank1 = 2.0 * d.c2[s.ref_gen] * s.base * s.base;

  // ---------------------------------------------------- evaluation gather
  // src = [LF (LF_STRIDE * nl) | u (nu) | pd (nb) | qd (nb)]
  s.src_u = LF_STRIDE * nl;
  const int src_pd = s.src_u + nu, src_qd = src_pd + nb;
  s.src_total = src_qd + nb;
  s.d_lu = 0;
  s.d_gu = s.d_lu + int(s.lu_col.size());
  s.d_a = s.d_gu + int(s.gu_col.size());
  s.d_g = s.d_a + int(s.a_col.size());
  s.d_h = s.d_g + nx;
  s.d_total = s.d_h + s.m;
  std::vector<std::vector<std::pair<int, double>>> terms(s.d_total);
  std::vector<double> cst(s.d_total, 0.0);
  auto jac_row = [&](int bus, bool isP, auto dst_of_w) {
    for (auto& le : ends[bus]) {
      int l = le.first, e = le.second;
      int base = isP ? (e == 0 ? LF_DPF : LF_DPT) : (e == 0 ? LF_DQF : LF_DQT);
      for (int kk = 0; kk < 4; ++kk) {
        int w = s.line_w[4 * l + kk];
        if (w < 0) continue;
        terms[dst_of_w(w)].push_back({(base + kk) * nl + l, 1.0});
      }
    }
  };
  auto value_sum = [&](int bus, bool isP, int dst) {
    for (auto& le : ends[bus]) {
      int l = le.first, e = le.second;
      int slot = isP ? (e == 0 ? LF_PF : LF_PT) : (e == 0 ? LF_QF : LF_QT);
      terms[dst].push_back({slot * nl + l, 1.0});
    }
  };
  for (int i = 0; i < nb; ++i) {
    for (int isP = 1; isP >= 0; --isP) {
      int nat = isP ? s.th_nat[i] : s.vmx_nat[i];
      if (nat < 0) continue;
      int ri = s.iperm[nat];
      jac_row(i, isP, [&](int w) {
        if (w >= nu) return s.d_lu + find_pos(s.lu_ptr, s.lu_col, ri, w - nu);
        return s.d_gu + find_pos(s.gu_ptr, s.gu_col, ri, w);
      });
      int gdst = s.d_g + nat;
      value_sum(i, isP, gdst);
      if (isP) {
        terms[gdst].push_back({src_pd + i, 1.0});
        int g = s.gen_of_bus[i];
        if (g >= 0 && s.pg_u[g] >= 0) {
          terms[gdst].push_back({s.src_u + s.pg_u[g], -1.0});
          cst[s.d_gu + find_pos(s.gu_ptr, s.gu_col, ri, s.pg_u[g])] = -1.0;
        }
      } else {
        terms[gdst].push_back({src_qd + i, 1.0});
      }
    }
  }
  auto arow_dst = [&](int row) {
    return [&, row](int w) { return s.d_a + find_pos(s.a_ptr, s.a_col, row, w); };
  };
  jac_row(s.ref, true, arow_dst(0));
  value_sum(s.ref, true, s.d_h + 0);
  terms[s.d_h + 0].push_back({src_pd + s.ref, 1.0});
  for (int g = 0; g < ng; ++g) {
    int b = d.gen_bus[g];
    jac_row(b, false, arow_dst(1 + g));
    value_sum(b, false, s.d_h + 1 + g);
    terms[s.d_h + 1 + g].push_back({src_qd + b, 1.0});
  }
  for (int l = 0; l < nl; ++l) {
    int kl = s.lim_of_line[l];
    if (kl < 0) continue;
    for (int e = 0; e < 2; ++e) {
      int row = 1 + ng + e * s.nlim + kl;
      for (int kk = 0; kk < 4; ++kk) {
        int w = s.line_w[4 * l + kk];
        if (w < 0) continue;
        terms[s.d_a + find_pos(s.a_ptr, s.a_col, row, w)].push_back(
            {((e == 0 ? LF_DSF2 : LF_DST2) + kk) * nl + l, 1.0});
      }
      terms[s.d_h + row].push_back({(e == 0 ? LF_SF2 : LF_ST2) * nl + l, 1.0});
    }
  }
  s.eg.ptr.assign(s.d_total + 1, 0);
  s.eg.idx.clear();
  s.eg.coef.clear();
  for (int e = 0; e < s.d_total; ++e) {
    for (auto& t : terms[e]) {
      s.eg.idx.push_back(t.first);
      s.eg.coef.push_back(t.second);
    }
    s.eg.ptr[e + 1] = int(s.eg.idx.size());
  }
  s.eg.cst = cst;
  return RH_OK;
}

// ------------------------------------------------------------------ checks
// A step list (4 ints per entry, the level third, the idle step last) as
// kCondWaves lists of one length, wave after wave: consecutive steps of one
// level go to the waves in turn, kCondWaves at a time (they touch distinct
// rows and read only rows of earlier levels), a wave with no step in a group
// takes the idle step, and every list ends with the idle step. Returns the
// number of groups.
int wave_groups(const Sweep& sw, int nwaves) {
  int groups = 0;
  for (int i = 0; i < sw.ks_nstep; ++groups) {
    int j = i;
    while (j < sw.ks_nstep && sw.ks_meta[size_t(kSweepMeta) * j + 3] == sw.ks_meta[size_t(kSweepMeta) * i + 3] &&
           j - i < nwaves)
      ++j;
    i = j;
  }
  return groups;
}

int group_for_waves(const int* e, size_t n_with_idle, int nwaves, std::vector<int>& out) {
  const size_t n = n_with_idle - 1;
  const int* idle = e + 4 * n;
  std::vector<std::vector<int>> lists(nwaves);
  int groups = 0;
  for (size_t i = 0; i < n; ++groups) {
    size_t j = i;
    while (j < n && e[4 * j + 2] == e[4 * i + 2] && j - i < size_t(nwaves)) ++j;
    for (int w = 0; w < nwaves; ++w) {
      const int* src = i + w < j ? e + 4 * (i + w) : idle;
      lists[w].insert(lists[w].end(), src, src + 4);
    }
    i = j;
  }
  for (auto& l : lists) {
    l.insert(l.end(), idle, idle + 4);
    out.insert(out.end(), l.begin(), l.end());
  }
  return groups;
}

void build_condense_records(const Symbolic& s, int W, CondenseRecords& R) {
  const long nw = s.nw, nu = s.nu;
  auto p_row = [&](long v) { return unsigned(v * W * 8); };                          // P row v
  auto h_row = [&](long v) { return unsigned(s.kst.pos[v] * W * 8); };   // H row v (over P)
  const Sweep* sws[4] = {&s.sl, &s.su, &s.sut, &s.slt};
  size_t nsteps = 0;
  for (auto* sw : sws) nsteps += size_t(sw->ks_nstep) + 1;
  R.steps.assign(nsteps * kStepDoubles, 0.0);
  R.tr_dst.clear();
  R.tr_src.clear();
  R.trd_dst.clear();
  R.trd_src.clear();
  size_t g = 0;
  for (int k = 0; k < 4; ++k) {
    const Sweep& sw = *sws[k];
    const bool on_h = k >= 2;   // U^T and L^T sweeps run on H
    R.meta[k].clear();
    for (int st = 0; st <= sw.ks_nstep; ++st, ++g) {
      const bool idle_step = st == sw.ks_nstep;
      const int* m = idle_step ? nullptr : &sw.ks_meta[size_t(kSweepMeta) * st];
      R.meta[k].insert(R.meta[k].end(), {int(g), idle_step ? 0 : m[2], idle_step ? -1 : m[3], 0});
      double* S = &R.steps[g * kStepDoubles];
      for (int t = 0; t < kSweepThreads; ++t) {
        // lanes past the step's rows take its padding block
        const int b = idle_step ? -1 : m[0] + std::min(t, m[1]);
        for (int j = 0; j < kSweepPF; ++j) {
          unsigned* off = reinterpret_cast<unsigned*>(S + (4 + j / 4) * kChunk + 2 * t);
          const size_t e = b >= 0 ? size_t(b) * kSweepPF + j : 0;
          const long row = nu + (b >= 0 ? sw.lb_col[e] : 0);
          off[j % 4] = on_h ? h_row(row) : p_row(row);
          if (b >= 0 && sw.lb_src[e] >= 0) {
            R.tr_dst.push_back(int(g * kStepDoubles + (j / 2) * kChunk + 2 * t + j % 2));
            R.tr_src.push_back(sw.lb_src[e]);
          }
        }
        double* piv = S + 6 * kChunk + 2 * t;
        unsigned* ro = reinterpret_cast<unsigned*>(piv + 1);
        const long row = nu + (b >= 0 ? sw.lb_row[b] : 0);
        ro[0] = on_h ? h_row(row) : p_row(row);
        ro[1] = b >= 0 && sw.lb_wr[b] ? 1u : 0u;
        if (ro[1] && sw.has_diag) {
          R.trd_dst.push_back(int(g * kStepDoubles + 6 * kChunk + 2 * t));
          R.trd_src.push_back(sw.lb_dsrc[b]);
        } else if (ro[1]) {
          *piv = 1.0;
        }
      }
    }
  }
  // Per column tile of the identity columns, the L-sweep steps that can
  // change its panel. Column j starts nonzero only in the rows of G_u's
  // column j, and a row turns nonzero only through a lower entry from a
  // nonzero row (the reach of those rows in the graph of L). A step whose
  // rows all lie outside the tile's reach subtracts zeros from zeros, so it
  // is left out and the results stay the same bit for bit. The tile holding
  // the right-hand-side column (a dense r4) keeps every step.
  {
    const int nx = s.nx;
    std::vector<std::vector<int>> lchild(nx);
    for (int i = 0; i < nx; ++i)
      for (int p = s.lu_ptr[i]; p < s.lu_diag[i]; ++p) lchild[s.lu_col[p]].push_back(i);
    const Sweep& sl = s.sl;
    std::vector<std::vector<int>> step_rows(sl.ks_nstep);
    for (int st = 0; st < sl.ks_nstep; ++st) {
      const int* m = &sl.ks_meta[size_t(kSweepMeta) * st];
      for (int t = 0; t < m[1]; ++t) step_rows[st].push_back(sl.lb_row[m[0] + t]);
    }
    const int ntile = int((nu + 1 + W - 1) / W);
    R.lsk_ptr.assign(ntile + 1, 0);
    R.lsk_meta.clear();
    std::vector<char> in(nx);
    std::vector<int> stack;
    for (int tile = 0; tile < ntile; ++tile) {
      const long j0 = long(tile) * W, j1 = std::min<long>(j0 + W, nu + 1);
      const bool full = j1 > nu;
      std::fill(in.begin(), in.end(), 0);
      if (!full) {
        for (long j = j0; j < j1; ++j)
          for (int e = s.gucsc_ptr[j]; e < s.gucsc_ptr[j + 1]; ++e) {
            const int r = s.gucsc_row[e];
            if (!in[r]) {
              in[r] = 1;
              stack.push_back(r);
            }
          }
        while (!stack.empty()) {
          const int k = stack.back();
          stack.pop_back();
          for (int i : lchild[k])
            if (!in[i]) {
              in[i] = 1;
              stack.push_back(i);
            }
        }
      }
      for (int st = 0; st < sl.ks_nstep; ++st) {
        bool need = full;
        for (int r : step_rows[st])
          if (in[r]) {
            need = true;
            break;
          }
        if (need)
          R.lsk_meta.insert(R.lsk_meta.end(), R.meta[0].begin() + 4 * size_t(st),
                            R.meta[0].begin() + 4 * size_t(st) + 4);
      }
      R.lsk_meta.insert(R.lsk_meta.end(), R.meta[0].end() - 4, R.meta[0].end());   // idle step
      R.lsk_ptr[tile + 1] = int(R.lsk_meta.size() / 4);
    }
    // the same lists for work-groups of several waves
    for (int c = 0; c < 2; ++c) {
      const int nwv = c ? kCondWavesWide : kCondWaves;
      R.lsk_gptr[c].assign(ntile + 1, 0);
      R.lsk_gmeta[c].clear();
      for (int tile = 0; tile < ntile; ++tile) {
        group_for_waves(&R.lsk_meta[4 * size_t(R.lsk_ptr[tile])],
                        size_t(R.lsk_ptr[tile + 1] - R.lsk_ptr[tile]), nwv, R.lsk_gmeta[c]);
        R.lsk_gptr[c][tile + 1] = int(R.lsk_gmeta[c].size() / 4);
      }
    }
  }
  for (int c = 0; c < 2; ++c)
    for (int k = 0; k < 4; ++k) {
      R.gmeta[c][k].clear();
      R.ngrp[c][k] = group_for_waves(R.meta[k].data(), R.meta[k].size() / 4,
                                     c ? kCondWavesWide : kCondWaves, R.gmeta[c][k]);
    }
  // record streams
  auto stream = [&](const Symbolic::LaneStream& ls, bool gt, std::vector<double>& str,
                    std::vector<int>& dst, std::vector<int>* xdst) {
    const size_t per = size_t(ls.nbat) * kStreamBatch;
    str.assign(size_t(ls.nbat) * kBatchDoubles, 0.0);
    for (int t = 0; t < kKRowBlock; ++t)
      for (size_t q = 0; q < per; ++q) {
        const size_t rec = t * per + q, i = q / kStreamBatch, r = q % kStreamBatch;
        const size_t vi = i * kBatchDoubles + (r / 2) * kChunk + 2 * t + r % 2;
        unsigned* off = reinterpret_cast<unsigned*>(&str[i * kBatchDoubles + (4 + r / 4) * kChunk + 2 * t]);
        const int kind = ls.kind[rec], c = ls.col[rec];
        if (kind == 0) {
          off[r % 4] = 0;
        } else if (!gt) {   // K: P rows (nw = the indicator row)
          off[r % 4] = p_row(c);
          (kind == 1 ? dst[ls.src[rec]] : (*xdst)[ls.src[rec]]) = int(vi);
        } else if (kind == 1) {   // G_u^T entry: H_x row
          off[r % 4] = h_row(nu + c);
          dst[ls.src[rec]] = int(vi);
        } else {   // -H_u of the row
          off[r % 4] = h_row(c);
          str[vi] = -1.0;
        }
      }
  };
  R.kdst.assign(std::max<size_t>(1, s.k_col.size()), 0);
  R.krt_dst.assign(size_t(nw), 0);
  R.gdst.assign(std::max<size_t>(1, s.gu_col.size()), 0);
  stream(s.kst, false, R.kstr, R.kdst, &R.krt_dst);
  stream(s.gst, true, R.gstr, R.gdst, nullptr);
  R.hpos = s.kst.pos;
  R.grow.assign(s.gst.row.begin(), s.gst.row.begin() + nu);
}

// Host refactorisation of G_x (values in natural CSR order) into LU
// positions, with the device's schedule (see host_solve).
rh_status host_refactor(const Symbolic& s, const double* gxv, std::vector<double>& lu_out) {
  const int nx = s.nx;
  std::vector<double>& lu = lu_out;
  lu.assign(s.lu_col.size(), 0.0);
  for (size_t p = 0; p < s.gx_col.size(); ++p) lu[s.gx_lu[p]] = gxv[p];
  // the device's static-pivot test: a pivot is too small when it is not
  // above 1e-14 times the largest entry of its row of G_x
  std::vector<double> rowmax(nx, 0.0);
  for (int i = 0; i < nx; ++i)
    for (int p = s.lu_ptr[i]; p < s.lu_ptr[i + 1]; ++p)
      rowmax[i] = std::max(rowmax[i], std::fabs(lu[p]));
  auto tiny = [&](int i, double piv) { return !(std::fabs(piv) > 1e-14 * rowmax[i]); };
  if (s.rw_ok) {
    // the wave-resident schedule, lane by lane as the device runs it
    std::vector<double> ulds(size_t(s.rw_nnz_u) + 1, 0.0), rinv(nx, 0.0);
    const int nlev = s.sl.nlev;
    for (int q = 0; q < s.sl.lev_ptr[1]; ++q) {            // level 0
      const int i = s.sl.rows[q];
      for (int p = s.lu_diag[i] + 1; p < s.lu_ptr[i + 1]; ++p)
        ulds[s.rw_ustart[i] + (p - s.lu_diag[i] - 1)] = lu[p];
      if (tiny(i, lu[s.lu_diag[i]])) return RH_SMALL_PIVOT;
      rinv[i] = 1.0 / lu[s.lu_diag[i]];
    }
    for (int lv = 0; lv < nlev; ++lv)
      for (int w = 0; w < kRwWaves; ++w) {
        const int k0 = lv ? s.rw_levend[size_t(w) * nlev + lv - 1] : 0;
        const int k1 = s.rw_levend[size_t(w) * nlev + lv];
        for (int k = k0; k < k1; ++k) {
          const int* R = &s.rw_rec[size_t(s.rw_wbeg[w] + k) * kRwRec];
          const int nsteps = R[1], wide = R[2];
          double acc[64], r[64];
          int ipos[64], pos[64], udst[64], drow[64];
          for (int ln = 0; ln < 64; ++ln) {
            const int seg = wide ? 0 : ln >> 4, p = wide ? ln : ln & 15;
            const int rp0 = R[4 + seg], len = R[8 + seg], nl = R[12 + seg];
            ipos[ln] = p < len ? rp0 + p : -1;
            acc[ln] = ipos[ln] >= 0 ? lu[ipos[ln]] : 0.0;
            r[ln] = p < nl ? rinv[s.lu_col[rp0 + p]] : 0.0;
            udst[ln] = p > nl && p < len ? R[16 + seg] + (p - nl - 1) : -1;
            drow[ln] = p == nl && p < len ? R[20 + seg] : -1;
            pos[ln] = p < nl ? p : -1;
          }
          for (int q = 0; q < nsteps; ++q) {
            double t[64];
            for (int ln = 0; ln < 64; ++ln) t[ln] = acc[ln] * r[ln];
            for (int ln = 0; ln < 64; ++ln) {
              const double l = wide ? t[q] : t[16 * (ln >> 4) + q];
              const unsigned pk = unsigned(s.rw_lane[size_t(R[0]) + size_t(q / 2) * 64 + ln]);
              const int ui = std::min(int((pk >> (16 * (q & 1))) & 0xffffu), s.rw_nnz_u);
              if (pos[ln] == q) acc[ln] = l;
              acc[ln] = std::fma(-l, ulds[ui], acc[ln]);
            }
          }
          for (int ln = 0; ln < 64; ++ln) {
            if (ipos[ln] >= 0) lu[ipos[ln]] = acc[ln];
            if (udst[ln] >= 0) ulds[udst[ln]] = acc[ln];
            if (drow[ln] >= 0) {
              if (tiny(drow[ln], acc[ln])) return RH_SMALL_PIVOT;
              rinv[drow[ln]] = 1.0 / acc[ln];
            }
          }
        }
      }
  } else
  // refactorise level by level (same schedule as the device)
  for (int lv = 0; lv < s.sl.nlev; ++lv)
    for (int sl = s.sl.lev_ptr[lv]; sl < s.sl.lev_ptr[lv + 1]; ++sl) {
      int i = s.sl.rows[sl];
      for (int p = s.lu_ptr[i]; p < s.lu_diag[i]; ++p) {
        double piv = lu[s.lu_diag[s.lu_col[p]]];
        if (piv == 0.0) return RH_SMALL_PIVOT;
        double l = lu[p] / piv;
        lu[p] = l;
        for (int o = s.rf_kptr[p]; o < s.rf_kptr[p + 1]; ++o) lu[s.rf_op_dst[o]] -= l * lu[s.rf_op_src[o]];
      }
    }
  for (int i = 0; i < nx; ++i)
    if (tiny(i, lu[s.lu_diag[i]])) return RH_SMALL_PIVOT;
  return RH_OK;
}

rh_status host_solve(const Symbolic& s, const double* gxv, const double* b, double* z,
                     bool transpose) {
  const int nx = s.nx;
  std::vector<double> lu;
  {
    const rh_status st = host_refactor(s, gxv, lu);
    if (st != RH_OK) return st;
  }
  for (int i = 0; i < nx; ++i)
    if (lu[s.lu_diag[i]] == 0.0) return RH_SMALL_PIVOT;
  std::vector<double> w(nx);
  for (int i = 0; i < nx; ++i) w[i] = b[s.perm[i]];
  // the sweeps follow the device's step schedule lane by lane: per lane an
  // FMA chain over its block, per row the DPP shift tree, then the writing
  // lane's (b - sum) * reciprocal pivot
  auto run = [&](const Sweep& sw) {
    for (int st = 0; st < sw.ks_nstep; ++st) {
      const int* m = &sw.ks_meta[size_t(kSweepMeta) * st];
      const int b0 = m[0], TL = m[1], S = 1 << m[2];
      std::vector<double> a(TL), out(TL);
      for (int t = 0; t < TL; ++t) {
        double acc = 0.0;
        for (int j = 0; j < kSweepPF; ++j) {
          const size_t e = size_t(b0 + t) * kSweepPF + j;
          const double v = sw.lb_src[e] >= 0 ? lu[sw.lb_src[e]] : 0.0;
          acc = std::fma(v, w[sw.lb_col[e]], acc);
        }
        a[t] = acc;
      }
      for (int g = 0; g < TL; g += S)
        for (int h = 1; h < S; h *= 2)
          for (int ln = S - 1; ln >= h; --ln) a[g + ln] += a[g + ln - h];
      for (int t = 0; t < TL; ++t)
        if (sw.lb_wr[b0 + t]) {
          const double dv = sw.has_diag ? 1.0 / lu[sw.lb_dsrc[b0 + t]] : 1.0;
          out[t] = (w[sw.lb_row[b0 + t]] - a[t]) * dv;
        }
      for (int t = 0; t < TL; ++t)
        if (sw.lb_wr[b0 + t]) w[sw.lb_row[b0 + t]] = out[t];
    }
  };
  if (!transpose) {
    run(s.sl);
    run(s.su);
  } else {
    run(s.sut);
    run(s.slt);
  }
  for (int i = 0; i < nx; ++i) z[s.perm[i]] = w[i];
  return RH_OK;
}

namespace {

// Dense solve A x = b (row-major n x n copy, partial pivoting).
void dense_solve(std::vector<double> A, int n, std::vector<double>& x) {
  for (int k = 0; k < n; ++k) {
    int pr = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[size_t(i) * n + k]) > std::fabs(A[size_t(pr) * n + k])) pr = i;
    if (pr != k) {
      for (int c = 0; c < n; ++c) std::swap(A[size_t(k) * n + c], A[size_t(pr) * n + c]);
      std::swap(x[k], x[pr]);
    }
    for (int i = k + 1; i < n; ++i) {
      const double f = A[size_t(i) * n + k] / A[size_t(k) * n + k];
      if (f == 0.0) continue;
      for (int c = k; c < n; ++c) A[size_t(i) * n + c] -= f * A[size_t(k) * n + c];
      x[i] -= f * x[k];
    }
  }
  for (int k = n - 1; k >= 0; --k) {
    double acc = x[k];
    for (int c = k + 1; c < n; ++c) acc -= A[size_t(k) * n + c] * x[c];
    x[k] = acc / A[size_t(k) * n + k];
  }
}

}  // namespace

rh_status host_check_condense(const Symbolic& s, int W, uint64_t seed, int ncols,
                              double* max_rel_err) {
  const int nx = s.nx, nu = s.nu, nw = s.nw;
  uint64_t st = seed * 6364136223846793005ull + 1442695040888963407ull;
  auto rnd = [&]() {   // uniform in [-1, 1)
    st = st * 6364136223846793005ull + 1442695040888963407ull;
    return double(st >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  };
  // values: G_x (natural CSR, dominant diagonal), G_u (CSR), K (CSR), rt, r4
  std::vector<double> gx(s.gx_col.size()), gu(s.gu_col.size()), kv(s.k_col.size()), rt(nw),
      r4(nx);
  for (int i = 0; i < nx; ++i) {
    double sum = 0.0;
    int dpos = -1;
    for (int p = s.gx_ptr[i]; p < s.gx_ptr[i + 1]; ++p) {
      gx[p] = rnd();
      sum += std::fabs(gx[p]);
      if (s.gx_col[p] == i) dpos = p;
    }
    if (dpos < 0) return RH_ERR_STATE;
    gx[dpos] = 2.0 + sum;
  }
  for (auto& v : gu) v = rnd();
  for (auto& v : kv) v = rnd();
  for (auto& v : rt) v = rnd();
  for (auto& v : r4) v = rnd();
  std::vector<double> lu;
  {
    const rh_status rs = host_refactor(s, gx.data(), lu);
    if (rs != RH_OK) return rs;
  }
  // device records with transcribed values
  CondenseRecords R;
  build_condense_records(s, W, R);
  for (size_t t = 0; t < R.tr_dst.size(); ++t) R.steps[R.tr_dst[t]] = lu[R.tr_src[t]];
  for (size_t t = 0; t < R.trd_dst.size(); ++t) R.steps[R.trd_dst[t]] = 1.0 / lu[R.trd_src[t]];
  for (size_t e = 0; e < s.k_col.size(); ++e) R.kstr[R.kdst[e]] = kv[e];
  for (int v = 0; v < nw; ++v) R.kstr[R.krt_dst[v]] = rt[v];
  for (size_t e = 0; e < s.gu_col.size(); ++e) R.gstr[R.gdst[e]] = gu[e];
  // dense references in the internal order (internal i <-> natural perm[i])
  std::vector<double> Gi(size_t(nx) * nx, 0.0), GiT(size_t(nx) * nx, 0.0);
  for (int r = 0; r < nx; ++r)
    for (int p = s.gx_ptr[r]; p < s.gx_ptr[r + 1]; ++p) {
      const int i = s.iperm[r], k = s.iperm[s.gx_col[p]];
      Gi[size_t(i) * nx + k] = gx[p];
      GiT[size_t(k) * nx + i] = gx[p];
    }
  double worst = 0.0;
  const int cols[3] = {0, nu / 2, nu};   // two control columns and the right-hand side
  for (int ci = 0; ci < std::min(ncols, 3); ++ci) {
    const int j = cols[ci];
    const bool rhs = j == nu;
    // ---- emulation of the condensation kernel for column 0 of a W-wide panel
    std::vector<double> pan(size_t(nw + 1) * W, 0.0), scr(size_t(nw) * W, 0.0);
    auto at = [&](unsigned off) -> double& { return pan[off / 8]; };
    if (rhs) {
      pan[size_t(nw) * W] = 1.0;
      for (int i = 0; i < nx; ++i) pan[size_t(nu + i) * W] = -r4[i];
    } else {
      pan[size_t(j) * W] = 1.0;
      for (int e = s.gucsc_ptr[j]; e < s.gucsc_ptr[j + 1]; ++e)
        pan[size_t(nu + s.gucsc_row[e]) * W] = -gu[s.gucsc_from_csr[e]];
    }
    for (int k = 0; k < 4; ++k) {
      const std::vector<int>& M = R.meta[k];
      const int n = int(M.size()) / 4 - 1;
      for (int q = 0; q < n; ++q) {
        const double* S = &R.steps[size_t(M[4 * q]) * kStepDoubles];
        const int ls = M[4 * q + 1];
        double a[kSweepThreads], xr[kSweepThreads];
        for (int t = 0; t < kSweepThreads; ++t) {
          double acc = 0.0;
          for (int jj = 0; jj < kSweepPF; ++jj) {
            const double v = S[(jj / 2) * kChunk + 2 * t + jj % 2];
            const unsigned o = reinterpret_cast<const unsigned*>(S + (4 + jj / 4) * kChunk + 2 * t)[jj % 4];
            acc = std::fma(v, at(o), acc);
          }
          a[t] = acc;
          xr[t] = at(reinterpret_cast<const unsigned*>(S + 6 * kChunk + 2 * t + 1)[0]);
        }
        for (int lv = 0; lv < std::min(ls, 4); ++lv) {   // DPP row shifts by 1, 2, 4, 8
          const int h = 1 << lv;
          double b2[kSweepThreads];
          for (int t = 0; t < kSweepThreads; ++t) b2[t] = a[t] + ((t % 16) >= h ? a[t - h] : 0.0);
          std::copy(b2, b2 + kSweepThreads, a);
        }
        if (ls >= 5) {
          double b2[kSweepThreads];
          for (int t = 0; t < kSweepThreads; ++t) {
            const int row = t / 16;
            b2[t] = a[t] + ((row == 1 || row == 3) ? a[16 * row - 1] : 0.0);
          }
          std::copy(b2, b2 + kSweepThreads, a);
        }
        if (ls >= 6) {
          double b2[kSweepThreads];
          for (int t = 0; t < kSweepThreads; ++t) b2[t] = a[t] + (t >= 32 ? a[31] : 0.0);
          std::copy(b2, b2 + kSweepThreads, a);
        }
        for (int t = 0; t < kSweepThreads; ++t) {
          const unsigned* ro = reinterpret_cast<const unsigned*>(S + 6 * kChunk + 2 * t + 1);
          if (ro[1]) at(ro[0]) = (xr[t] - a[t]) * S[6 * kChunk + 2 * t];
        }
      }
      if (k == 1) {   // H = K [V; Z] after the L and U sweeps
        const Symbolic::LaneStream& ls = s.kst;
        for (int t = 0; t < kKRowBlock; ++t) {
          double acc = 0.0;
          int b = 0;
          for (int q = 0; q < ls.end.back(); ++q) {
            const size_t i = q / kStreamBatch, r = q % kStreamBatch;
            const double v = R.kstr[i * kBatchDoubles + (r / 2) * kChunk + 2 * t + r % 2];
            const unsigned o = reinterpret_cast<const unsigned*>(&R.kstr[i * kBatchDoubles + (4 + r / 4) * kChunk + 2 * t])[r % 4];
            acc = std::fma(v, at(o), acc);
            while (b < int(ls.end.size()) && q + 1 == ls.end[b]) {
              const int p = b * kKRowBlock + t;
              if (p < nw) scr[size_t(p) * W] = acc;
              acc = 0.0;
              ++b;
            }
          }
        }
        for (int p = 0; p < nw; ++p) pan[size_t(p) * W] = scr[size_t(p) * W];   // H over P
      }
    }
    std::vector<double> out(nu);
    {
      const Symbolic::LaneStream& ls = s.gst;
      for (int t = 0; t < kKRowBlock; ++t) {
        double acc = 0.0;
        int b = 0;
        for (int q = 0; q < (ls.end.empty() ? 0 : ls.end.back()); ++q) {
          const size_t i = q / kStreamBatch, r = q % kStreamBatch;
          const double v = R.gstr[i * kBatchDoubles + (r / 2) * kChunk + 2 * t + r % 2];
          const unsigned o = reinterpret_cast<const unsigned*>(&R.gstr[i * kBatchDoubles + (4 + r / 4) * kChunk + 2 * t])[r % 4];
          acc = std::fma(v, at(o), acc);
          while (b < int(ls.end.size()) && q + 1 == ls.end[b]) {
            const int p = b * kKRowBlock + t;
            if (p < nu) out[R.grow[p]] = -acc;
            acc = 0.0;
            ++b;
          }
        }
      }
    }
    // ---- dense reference
    std::vector<double> z(nx, 0.0);
    if (rhs) {
      for (int i = 0; i < nx; ++i) z[i] = -r4[i];
    } else {
      for (int i = 0; i < nx; ++i)
        for (int e = s.gu_ptr[i]; e < s.gu_ptr[i + 1]; ++e)
          if (s.gu_col[e] == j) z[i] -= gu[e];
    }
    dense_solve(Gi, nx, z);
    std::vector<double> w(nw, 0.0), hcol(nw, 0.0);
    if (!rhs) w[j] = 1.0;
    for (int i = 0; i < nx; ++i) w[nu + i] = z[i];
    for (int v = 0; v < nw; ++v) {
      double acc = rhs ? rt[v] : 0.0;
      for (int p = s.k_ptr[v]; p < s.k_ptr[v + 1]; ++p) acc += kv[p] * w[s.k_col[p]];
      hcol[v] = acc;
    }
    std::vector<double> psi(hcol.begin() + nu, hcol.end());
    dense_solve(GiT, nx, psi);
    double scale = 0.0, err = 0.0;
    for (int q = 0; q < nu; ++q) {
      double ref = hcol[q];
      for (int i = 0; i < nx; ++i)
        for (int e = s.gu_ptr[i]; e < s.gu_ptr[i + 1]; ++e)
          if (s.gu_col[e] == q) ref -= gu[e] * psi[i];
      scale = std::max(scale, std::fabs(ref));
      err = std::max(err, std::fabs(ref - out[q]));
    }
    worst = std::max(worst, err / std::max(scale, 1e-300));
  }
  *max_rel_err = worst;
  return RH_OK;
}

rh_status check_levels(const Symbolic& s) {
  for (const Sweep* sw : {&s.sl, &s.su, &s.sut, &s.slt}) {
    std::vector<int> lv(s.nx, -1);
    for (int l = 0; l < sw->nlev; ++l)
      for (int q = sw->lev_ptr[l]; q < sw->lev_ptr[l + 1]; ++q) {
        if (lv[sw->rows[q]] != -1) return RH_ERR_STATE;
        lv[sw->rows[q]] = l;
      }
    for (int i = 0; i < s.nx; ++i)
      if (lv[i] < 0) return RH_ERR_STATE;
    std::vector<int> slot_of(s.nx, -1);
    for (int l = 0; l < sw->nlev; ++l)
      for (int q = sw->lev_ptr[l]; q < sw->lev_ptr[l + 1]; ++q) {
        slot_of[sw->rows[q]] = q;
        for (int e = sw->ptr[q]; e < sw->ptr[q + 1]; ++e)
          if (lv[sw->col[e]] >= l) return RH_ERR_STATE;
      }
    // step schedule: shapes, every row with work written by exactly one
    // lane, each group's lanes on one row with exactly the row's entries,
    // every column read finished in an earlier step (or never written: a
    // unit-diagonal row with no entries), idle blocks all padding
    std::vector<int> step_of(s.nx, -1);
    for (int st = 0; st < sw->ks_nstep; ++st) {
      const int* m = &sw->ks_meta[size_t(kSweepMeta) * st];
      const int b0 = m[0], TL = m[1], ls = m[2], S = 1 << ls;
      if (ls < 0 || S > kSweepMaxLanes || TL < S || TL % S || TL > kSweepThreads)
        return RH_ERR_STATE;
      if (b0 < 0 || b0 + TL + 1 > sw->lb_n || (st + 1 < sw->ks_nstep && sw->ks_meta[size_t(kSweepMeta) * (st + 1)] != b0 + TL + 1))
        return RH_ERR_STATE;
      for (int t = 0; t < TL; t += S) {
        const int i = sw->lb_row[b0 + t];
        if (i < 0 || i >= s.nx || step_of[i] != -1) return RH_ERR_STATE;
        step_of[i] = st;
        for (int k = 0; k < S; ++k)
          if (sw->lb_row[b0 + t + k] != i || sw->lb_wr[b0 + t + k] != (k == S - 1 ? 1 : 0))
            return RH_ERR_STATE;
        if (sw->has_diag && sw->lb_dsrc[b0 + t + S - 1] != sw->diag_src[slot_of[i]])
          return RH_ERR_STATE;
      }
      const int idle = b0 + TL;
      if (sw->lb_wr[idle] != 0) return RH_ERR_STATE;
      for (int j = 0; j < kSweepPF; ++j)
        if (sw->lb_src[size_t(idle) * kSweepPF + j] != -1) return RH_ERR_STATE;
    }
    for (int i = 0; i < s.nx; ++i) {
      const int q = slot_of[i];
      const bool work = sw->has_diag || sw->ptr[q + 1] > sw->ptr[q];
      if ((step_of[i] >= 0) != work) return RH_ERR_STATE;
    }
    // the step lists of work-groups of several waves: NW lists of ngrp + 1
    // entries each ending with the idle step; group g holds, wave by wave,
    // the next steps of the schedule, all of one level (so none reads a row
    // another writes), idle steps after them; every step exactly once
    for (const int nwv : {kCondWaves, kCondWavesWide}) {
      std::vector<int> e;
      for (int st = 0; st < sw->ks_nstep; ++st)
        e.insert(e.end(), {st, sw->ks_meta[size_t(kSweepMeta) * st + 2],
                           sw->ks_meta[size_t(kSweepMeta) * st + 3], 0});
      e.insert(e.end(), {sw->ks_nstep, 0, -1, 0});
      std::vector<int> out;
      const int G = group_for_waves(e.data(), e.size() / 4, nwv, out);
      if (G != wave_groups(*sw, nwv) || out.size() != size_t(4) * nwv * (G + 1))
        return RH_ERR_STATE;
      auto at = [&](int w, int g) { return &out[4 * (size_t(w) * (G + 1) + g)]; };
      int next = 0;
      for (int g = 0; g <= G; ++g) {
        int lev = -2;
        bool idle_seen = false;
        for (int w = 0; w < nwv; ++w) {
          const int* m = at(w, g);
          if (m[0] == sw->ks_nstep) {   // idle
            if (m[2] != -1) return RH_ERR_STATE;
            idle_seen = true;
            continue;
          }
          if (g == G || idle_seen || m[0] != next) return RH_ERR_STATE;
          if (lev != -2 && m[2] != lev) return RH_ERR_STATE;
          lev = m[2];
          ++next;
        }
        if (g < G && lev == -2) return RH_ERR_STATE;   // an empty group
      }
      if (next != sw->ks_nstep) return RH_ERR_STATE;
    }
    for (int st = 0; st < sw->ks_nstep; ++st) {
      const int* m = &sw->ks_meta[size_t(kSweepMeta) * st];
      const int b0 = m[0], TL = m[1], S = 1 << m[2];
      for (int t = 0; t < TL; t += S) {
        const int i = sw->lb_row[b0 + t], q = slot_of[i];
        std::vector<std::pair<int, int>> got, want;
        for (int k = 0; k < S; ++k)
          for (int j = 0; j < kSweepPF; ++j) {
            const size_t e = size_t(b0 + t + k) * kSweepPF + j;
            if (sw->lb_src[e] >= 0) got.push_back({sw->lb_col[e], sw->lb_src[e]});
          }
        for (int e = sw->ptr[q]; e < sw->ptr[q + 1]; ++e) want.push_back({sw->col[e], sw->src[e]});
        std::sort(got.begin(), got.end());
        std::sort(want.begin(), want.end());
        if (got != want) return RH_ERR_STATE;
        for (auto& ce : got)
          if (step_of[ce.first] >= st) return RH_ERR_STATE;
      }
    }
  }
  // wave-resident refactorisation: every task's global U positions (read by
  // the per-level launches) name the same U entries as its packed LDS slots,
  // and the split levels are a prefix of the L levels
  if (s.rw_ok) {
    if (s.rw_split < 0 || s.rw_split >= s.sl.nlev) return RH_ERR_STATE;
    std::vector<int> slot_lu(size_t(s.rw_nnz_u) + 1, -1);
    for (int i = 0; i < s.nx; ++i)
      for (int p = s.lu_diag[i] + 1; p < s.lu_ptr[i + 1]; ++p)
        slot_lu[size_t(s.rw_ustart[i]) + (p - s.lu_diag[i] - 1)] = p;
    const int ntask = int(s.rw_rec.size()) / kRwRec - 1;
    for (int k = 0; k < ntask; ++k) {
      const int* rec = &s.rw_rec[size_t(k) * kRwRec];
      const int off = rec[0], nsteps = rec[1], lu0 = rec[3];
      if (lu0 < 0 || size_t(lu0) + size_t(nsteps) * 64 > s.rw_lanelu.size()) return RH_ERR_STATE;
      for (int q = 0; q < nsteps; ++q)
        for (int lane = 0; lane < 64; ++lane) {
          const unsigned pk = unsigned(s.rw_lane[size_t(off) + size_t(q / 2) * 64 + lane]);
          const int ui = int((pk >> (16 * (q & 1))) & 0xffffu);
          const int want = ui >= s.rw_nnz_u ? -1 : slot_lu[ui];
          if (s.rw_lanelu[size_t(lu0) + size_t(q) * 64 + lane] != want) return RH_ERR_STATE;
        }
    }
  }
  return RH_OK;
}

}  // namespace rh
