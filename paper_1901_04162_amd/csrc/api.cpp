// C-ABI entry points and host-side mesh planning of libmomfill.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "internal.hpp"

namespace mf {

static thread_local std::string g_err;

void set_error(const std::string &msg) { g_err = msg; }

int hip_fail(hipError_t e, const char *what) {
  set_error(std::string("HIP error ") + hipGetErrorString(e) + " in " + what);
  return MF_EHIP;
}

static int fail(int code, const std::string &msg) {
  set_error(msg);
  return code;
}

// Symmetric triangle rules of degree 2, 4 and 5 (barycentric, weights sum
// to one); coordinates and weights of the 6-point rule from their closed
// forms.
bool make_rule(int q, Rule *r) {
  auto put = [&](int i, double a, double b, double c) {
    r->bary[i][0] = a;
    r->bary[i][1] = b;
    r->bary[i][2] = c;
  };
  if (q == 3) {
    const double a = 2.0 / 3.0, b = 1.0 / 6.0;
    put(0, a, b, b);
    put(1, b, a, b);
    put(2, b, b, a);
    r->w[0] = r->w[1] = r->w[2] = 1.0 / 3.0;
  } else if (q == 6) {
    const double s10 = std::sqrt(10.0);
    const double rt = std::sqrt(38.0 - 44.0 * std::sqrt(2.0 / 5.0));
    const double a1 = (8.0 - s10 + rt) / 18.0, a2 = (8.0 - s10 - rt) / 18.0;
    const double wr = std::sqrt(213125.0 - 53320.0 * s10);
    const double w1 = (620.0 + wr) / 3720.0, w2 = (620.0 - wr) / 3720.0;
    const double b1 = 1.0 - 2.0 * a1, b2 = 1.0 - 2.0 * a2;
    put(0, b1, a1, a1);
    put(1, a1, b1, a1);
    put(2, a1, a1, b1);
    put(3, b2, a2, a2);
    put(4, a2, b2, a2);
    put(5, a2, a2, b2);
    r->w[0] = r->w[1] = r->w[2] = w1;
    r->w[3] = r->w[4] = r->w[5] = w2;
  } else if (q == 7) {
    const double s15 = std::sqrt(15.0);
    const double a = (6.0 - s15) / 21.0, b = (9.0 + 2.0 * s15) / 21.0;
    const double c = (6.0 + s15) / 21.0, d = (9.0 - 2.0 * s15) / 21.0;
    put(0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 3.0);
    put(1, b, a, a);
    put(2, a, b, a);
    put(3, a, a, b);
    put(4, d, c, c);
    put(5, c, d, c);
    put(6, c, c, d);
    r->w[0] = 9.0 / 40.0;
    r->w[1] = r->w[2] = r->w[3] = (155.0 - s15) / 1200.0;
    r->w[4] = r->w[5] = r->w[6] = (155.0 + s15) / 1200.0;
  } else {
    return false;
  }
  r->nq = q;
  return true;
}

// ---- mesh planning --------------------------------------------------------

struct HalfEdge {
  int lo, hi, t, a;
  bool up;
};

static int build_topology(mf_mesh *m) {
  const int nt = m->nt, nv = m->nv;
  std::vector<HalfEdge> h(3 * (size_t)nt);
  for (int t = 0; t < nt; ++t) {
    const int32_t *v = &m->tri[3 * (size_t)t];
    for (int c = 0; c < 3; ++c)
      if (v[c] < 0 || v[c] >= nv) return fail(MF_EMESH, "vertex index out of range");
    if (v[0] == v[1] || v[1] == v[2] || v[0] == v[2])
      return fail(MF_EMESH, "triangle with a repeated vertex");
    for (int a = 0; a < 3; ++a) {
      int from = v[(a + 1) % 3], to = v[(a + 2) % 3];
      h[3 * (size_t)t + a] = {std::min(from, to), std::max(from, to), t, a, from < to};
    }
  }
  std::vector<uint32_t> idx(h.size());
  for (size_t i = 0; i < idx.size(); ++i) idx[i] = (uint32_t)i;
  std::sort(idx.begin(), idx.end(), [&](uint32_t x, uint32_t y) {
    if (h[x].lo != h[y].lo) return h[x].lo < h[y].lo;
    if (h[x].hi != h[y].hi) return h[x].hi < h[y].hi;
    return x < y;
  });
  // interior edges keyed by first appearance (3t + a of the earlier half-edge)
  std::vector<std::pair<uint32_t, uint32_t>> interior;  // (first, group start)
  for (size_t i = 0; i < idx.size();) {
    size_t j = i;
    while (j < idx.size() && h[idx[j]].lo == h[idx[i]].lo && h[idx[j]].hi == h[idx[i]].hi) ++j;
    if (j - i > 2) return fail(MF_EMESH, "edge shared by more than two triangles");
    if (j - i == 2) {
      if (h[idx[i]].up == h[idx[i + 1]].up)
        return fail(MF_EMESH, "inconsistently oriented neighbouring triangles");
      interior.push_back({std::min(idx[i], idx[i + 1]), (uint32_t)i});
    }
    i = j;
  }
  std::sort(interior.begin(), interior.end());
  m->ne = (int)interior.size();
  m->edges.assign(6 * (size_t)m->ne, 0);
  m->tedge.assign(3 * (size_t)nt, -1);
  m->tsign.assign(3 * (size_t)nt, 0);
  for (int e = 0; e < m->ne; ++e) {
    const HalfEdge &x = h[idx[interior[e].second]], &y = h[idx[interior[e].second + 1]];
    const HalfEdge &pl = x.up ? x : y, &mi = x.up ? y : x;
    int32_t *E = &m->edges[6 * (size_t)e];
    E[0] = x.lo;
    E[1] = x.hi;
    E[2] = pl.t;
    E[3] = mi.t;
    E[4] = pl.a;
    E[5] = mi.a;
    m->tedge[3 * (size_t)pl.t + pl.a] = e;
    m->tsign[3 * (size_t)pl.t + pl.a] = 1;
    m->tedge[3 * (size_t)mi.t + mi.a] = e;
    m->tsign[3 * (size_t)mi.t + mi.a] = -1;
  }
  if (m->ne == 0) return fail(MF_EMESH, "mesh has no interior edge");
  return MF_OK;
}

static void build_touching(mf_mesh *m) {
  const int nt = m->nt;
  std::vector<std::vector<int32_t>> vt(m->nv);
  for (int t = 0; t < nt; ++t)
    for (int c = 0; c < 3; ++c) vt[m->tri[3 * (size_t)t + c]].push_back(t);
  m->touch_off.assign(nt + 1, 0);
  m->touch_q.clear();
  std::vector<int32_t> nb;
  for (int p = 0; p < nt; ++p) {
    nb.clear();
    for (int c = 0; c < 3; ++c)
      for (int32_t q : vt[m->tri[3 * (size_t)p + c]]) nb.push_back(q);
    std::sort(nb.begin(), nb.end());
    nb.erase(std::unique(nb.begin(), nb.end()), nb.end());
    m->touch_q.insert(m->touch_q.end(), nb.begin(), nb.end());
    m->touch_off[p + 1] = (int32_t)m->touch_q.size();
  }
  m->touch_rev.assign(m->touch_q.size(), -1);
  for (int p = 0; p < nt; ++p)
    for (int32_t s = m->touch_off[p]; s < m->touch_off[p + 1]; ++s) {
      const int q = m->touch_q[s];
      auto b = m->touch_q.begin() + m->touch_off[q], e = m->touch_q.begin() + m->touch_off[q + 1];
      m->touch_rev[s] = (int32_t)(std::lower_bound(b, e, p) - m->touch_q.begin());
    }
  m->touch_p.resize(m->touch_q.size());
  m->touch_u.clear();
  for (int p = 0; p < nt; ++p)
    for (int32_t s = m->touch_off[p]; s < m->touch_off[p + 1]; ++s) {
      m->touch_p[s] = p;
      if (p <= m->touch_q[s]) m->touch_u.push_back(s);
    }
}

// Rounds of a block's source triangles for an accumulation without atomics:
// at most cap triangles per round and no two of a round adjacent (sharing an
// edge), so no two waves add to one column at once.  adj[3 i + a] is the
// local index of triangle i's neighbour across its edge a inside the block, or
// -1.  First fit over a few orders: the two classes of a breadth-first
// two-colouring of the adjacency (a triangulated patch is mostly bipartite,
// then the rounds come out full), index order, and seeded shuffles; the order
// with the fewest rounds wins.  order receives the local indices in round
// order, starts the maxr + 1 round starts; false when more than maxr rounds
// would be needed.
static bool block_rounds(const std::vector<int> &adj, int n, int cap, int maxr, int32_t *order,
                         int32_t *starts, uint64_t &seed) {
  std::vector<int> par(n, -1), round_of(n, -1), best_round(n, -1), cnt(maxr, 0);
  std::vector<int32_t> ord, queue;
  for (int s0 = 0; s0 < n; ++s0) {  // two-colouring, breadth first
    if (par[s0] >= 0) continue;
    par[s0] = 0;
    queue.assign(1, s0);
    for (size_t h = 0; h < queue.size(); ++h)
      for (int a = 0; a < 3; ++a) {
        const int o = adj[3 * (size_t)queue[h] + a];
        if (o >= 0 && par[o] < 0) {
          par[o] = 1 - par[queue[h]];
          queue.push_back(o);
        }
      }
  }
  auto first_fit = [&](const std::vector<int32_t> &o) -> int {
    std::fill(cnt.begin(), cnt.end(), 0);
    int nr = 0;
    for (int t : o) round_of[t] = -1;
    for (int t : o) {
      int r = 0;
      for (; r < maxr; ++r) {
        if (cnt[r] >= cap) continue;
        bool clash = false;
        for (int a = 0; a < 3 && !clash; ++a) {
          const int nb = adj[3 * (size_t)t + a];
          clash = nb >= 0 && round_of[nb] == r;
        }
        if (!clash) break;
      }
      if (r == maxr) return maxr + 1;
      round_of[t] = r;
      ++cnt[r];
      nr = std::max(nr, r + 1);
    }
    return nr;
  };
  const int ideal = (n + cap - 1) / cap;
  int best = maxr + 1;
  for (int trial = 0; trial < 36 && best > ideal; ++trial) {
    ord.resize(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    if (trial < 2)
      std::stable_sort(ord.begin(), ord.end(),
                       [&](int x, int y) { return (par[x] ^ trial) < (par[y] ^ trial); });
    else if (trial > 2)
      for (int i = n - 1; i > 0; --i) {  // seeded shuffle
        seed = seed * 6364136223846793005ull + 1442695040888963407ull;
        std::swap(ord[i], ord[(int)((seed >> 33) % (uint64_t)(i + 1))]);
      }
    const int nr = first_fit(ord);
    if (nr < best) {
      best = nr;
      best_round = round_of;
    }
  }
  if (best > maxr) return false;
  int pos = 0;
  for (int r = 0; r <= maxr; ++r) {
    starts[r] = pos;
    if (r < best)
      for (int t = 0; t < n; ++t)
        if (best_round[t] == r) order[pos++] = t;
  }
  return true;
}

// Row/column blocks of the tiled fill: runs of consecutive edges (so every
// tile is a contiguous rectangle of Z) carrying at most kMaxBlockTris
// triangles and kMaxBlockEdges edges.  Boundaries come from a dynamic program
// that minimises the number of distinct triangles summed over blocks plus a
// per-block cost: every triangle in a block is recomputed by each tile of
// that block row, so fewer distinct triangles means less repeated work.
static void build_blocks(mf_mesh *m) {
  const int ne = m->ne;
  const int32_t *E = m->edges.data();
  const double kBlockCost = 32.0;
  std::vector<double> best(ne + 1, 1e300);
  std::vector<int32_t> from(ne + 1, 0), stamp(m->nt, -1);
  best[0] = 0.0;
  for (int e = 1; e <= ne; ++e) {
    int ntri = 0;
    for (int len = 1; len <= kMaxBlockEdges && e - len >= 0; ++len) {
      const int s = e - len;
      for (int c = 2; c <= 3; ++c) {
        const int t = E[6 * (size_t)s + c];
        if (stamp[t] != e) {
          stamp[t] = e;
          ++ntri;
        }
      }
      if (ntri > kMaxBlockTris) break;
      const double cost = best[s] + ntri + kBlockCost;
      if (cost < best[e]) {
        best[e] = cost;
        from[e] = s;
      }
    }
  }
  std::vector<int32_t> starts;
  for (int e = ne; e > 0; e = from[e]) starts.push_back(from[e]);
  std::reverse(starts.begin(), starts.end());
  m->nblk = (int)starts.size();
  m->blk_e0 = starts;
  m->blk_e0.push_back(ne);
  m->blk_off.assign(m->nblk + 1, 0);
  m->blk_tri.clear();
  m->blk_pos.clear();
  m->blk_rt.assign((size_t)m->nblk * kMaxBlockEdges, 0);
  m->max_blk_tris = 0;
  std::vector<int32_t> tl;
  for (int b = 0; b < m->nblk; ++b) {
    const int e0 = m->blk_e0[b], e1 = m->blk_e0[b + 1];
    tl.clear();
    for (int e = e0; e < e1; ++e) {
      tl.push_back(E[6 * (size_t)e + 2]);
      tl.push_back(E[6 * (size_t)e + 3]);
    }
    std::sort(tl.begin(), tl.end());
    tl.erase(std::unique(tl.begin(), tl.end()), tl.end());
    for (int32_t t : tl) {
      uint32_t pk = 0;
      for (int a = 0; a < 3; ++a) {
        const int e = m->tedge[3 * (size_t)t + a];
        const uint32_t pos = (e >= e0 && e < e1) ? (uint32_t)(e - e0) : 0xffu;
        pk |= pos << (8 * a);
      }
      m->blk_tri.push_back(t);
      m->blk_pos.push_back((int32_t)pk);
    }
    for (int e = e0; e < e1; ++e) {
      const auto pos = [&](int32_t t) {
        return (int32_t)(std::lower_bound(tl.begin(), tl.end(), t) - tl.begin());
      };
      m->blk_rt[(size_t)b * kMaxBlockEdges + (e - e0)] =
          pos(E[6 * (size_t)e + 2]) | (pos(E[6 * (size_t)e + 3]) << 8);
    }
    m->blk_off[b + 1] = (int32_t)m->blk_tri.size();
    m->max_blk_tris = std::max(m->max_blk_tris, (int)tl.size());
  }
  // rounds of each edge block's triangles (block_rounds), for the MFIE tile,
  // which accumulates both directions of a pair without atomics: blk_ord holds
  // positions in the block's triangle list, in round order
  m->blk_ord.assign(m->blk_tri.size(), 0);
  m->blk_rounds.assign((size_t)m->nblk * (kEBMaxRounds + 1), 0);
  {
    std::vector<int> adj, pos_of(m->nt, -1);
    uint64_t seed = 0x2545f4914f6cdd1dull;
    for (int b = 0; b < m->nblk; ++b) {
      const int p0 = m->blk_off[b], n = m->blk_off[b + 1] - p0;
      for (int i = 0; i < n; ++i) pos_of[m->blk_tri[p0 + i]] = i;
      adj.assign(3 * (size_t)n, -1);
      for (int i = 0; i < n; ++i) {
        const int t = m->blk_tri[p0 + i];
        for (int a = 0; a < 3; ++a) {
          const int e = m->tedge[3 * (size_t)t + a];
          if (e < 0) continue;
          const int o = E[6 * (size_t)e + 2] == t ? E[6 * (size_t)e + 3] : E[6 * (size_t)e + 2];
          adj[3 * (size_t)i + a] = pos_of[o];
        }
      }
      // at most 3 neighbours each: first fit never needs more than
      // n / kEBRound + 4 rounds, within kEBMaxRounds for n <= kMaxBlockTris
      block_rounds(adj, n, kEBRound, kEBMaxRounds, &m->blk_ord[p0],
                   &m->blk_rounds[(size_t)b * (kEBMaxRounds + 1)], seed);
      for (int i = 0; i < n; ++i) pos_of[m->blk_tri[p0 + i]] = -1;
    }
  }
  // Z is symmetric (Galerkin reciprocity): only block pairs I <= J are filled.
  // Tiles pack I and J into 16 bits each (unsigned); with at most 65535
  // blocks there are fewer than 2^31 tiles.  Larger plans are refused by the
  // caller before any tile is listed.
  m->tiles.clear();
  if (m->nblk > 65535) return;
  for (int I = 0; I < m->nblk; ++I)
    for (int J = I; J < m->nblk; ++J) m->tiles.push_back((int32_t)(((uint32_t)I << 16) | (uint32_t)J));
}

// Triangle-block plan of the table-mode fill.  Blocks are runs of
// consecutive triangles (at most kTBTris), closed before their block-edge
// count would pass kTBEdges.  Edges are numbered by first appearance, so the
// edges a block owns (first seen in its triangles) form one run of edge ids.
// An edge with its two triangles in different blocks is cut: the block of
// its lower triangle owns it, the other holds its non-owner half.  The
// source triangles of each block are put in rounds of at most kTBRound
// triangles of which no two share an edge (greedy, in index order).
static void build_tb_plan(mf_mesh *m) {
  m->tb_ok = false;
  const int nt = m->nt, ne = m->ne;
  const int32_t *E = m->edges.data();
  std::vector<int32_t> blk(nt, -1);
  m->tb_t0.assign(1, 0);
  {
    int t0 = 0, cnt = 0;
    for (int t = 0; t < nt; ++t) {
      int add = 0;
      for (int a = 0; a < 3; ++a) {
        const int e = m->tedge[3 * (size_t)t + a];
        if (e < 0) continue;
        const int o = E[6 * (size_t)e + 2] == t ? E[6 * (size_t)e + 3] : E[6 * (size_t)e + 2];
        if (!(o >= t0 && o < t)) ++add;
      }
      if (t > t0 && (t - t0 == kTBTris || cnt + add > kTBEdges)) {
        m->tb_t0.push_back(t);
        t0 = t;
        cnt = 0;
        add = 0;
        for (int a = 0; a < 3; ++a) add += m->tedge[3 * (size_t)t + a] >= 0;
      }
      if (add > kTBEdges) return;  // cannot happen for triangles (at most 3 edges)
      cnt += add;
      blk[t] = (int)m->tb_t0.size() - 1;
    }
    m->tb_t0.push_back(nt);
  }
  const int nb = (int)m->tb_t0.size() - 1;
  if (nb > 65535) return;
  m->tb_nblk = nb;
  // owned edge runs, cut indices
  m->tb_e0.assign(nb + 1, ne);
  m->cut_idx.assign(ne, -1);
  m->cut_edge.clear();
  for (int e = ne - 1; e >= 0; --e) {
    const int tp = E[6 * (size_t)e + 2], tm = E[6 * (size_t)e + 3];
    m->tb_e0[blk[std::min(tp, tm)]] = e;
  }
  for (int b = nb - 1; b >= 0; --b)
    if (m->tb_e0[b] > m->tb_e0[b + 1]) m->tb_e0[b] = m->tb_e0[b + 1];  // a block owning none
  for (int e = 0; e < ne; ++e) {
    const int tp = E[6 * (size_t)e + 2], tm = E[6 * (size_t)e + 3];
    const int lo = std::min(tp, tm);
    if (e < m->tb_e0[blk[lo]] || e >= m->tb_e0[blk[lo] + 1]) return;  // runs must hold
    if (blk[tp] != blk[tm]) {
      m->cut_idx[e] = (int)m->cut_edge.size();
      m->cut_edge.push_back(e);
    }
  }
  m->n_cut = (int)m->cut_edge.size();
  // non-owner halves per block (in edge order) and their local indices
  std::vector<std::vector<int32_t>> half(nb);
  for (int e = 0; e < ne; ++e) {
    if (m->cut_idx[e] < 0) continue;
    const int hi = std::max(E[6 * (size_t)e + 2], E[6 * (size_t)e + 3]);
    half[blk[hi]].push_back(e);
  }
  m->tb_nbe.assign(nb, 0);
  m->tb_be_off.assign(nb + 1, 0);
  m->tb_be_cut.clear();
  std::vector<int32_t> local(ne, -1);  // local index of a non-owner half in its block
  for (int b = 0; b < nb; ++b) {
    const int nown = m->tb_e0[b + 1] - m->tb_e0[b];
    for (size_t k = 0; k < half[b].size(); ++k) {
      local[half[b][k]] = nown + (int)k;
      m->tb_be_cut.push_back(m->cut_idx[half[b][k]]);
    }
    m->tb_nbe[b] = nown + (int)half[b].size();
    m->tb_be_off[b + 1] = (int32_t)m->tb_be_cut.size();
    if (m->tb_nbe[b] > kTBEdges) return;
  }
  m->tb_pos.assign(nt, -1);
  for (int t = 0; t < nt; ++t) {
    const int b = blk[t];
    uint32_t pk = 0;
    for (int a = 0; a < 3; ++a) {
      const int e = m->tedge[3 * (size_t)t + a];
      uint32_t r = 0xffu;
      if (e >= 0) r = (e >= m->tb_e0[b] && e < m->tb_e0[b + 1]) ? (uint32_t)(e - m->tb_e0[b])
                                                                   : (uint32_t)local[e];
      pk |= r << (8 * a);
    }
    m->tb_pos[t] = (int32_t)pk;
  }
  // rounds of each block's triangles (block_rounds)
  m->tb_order.assign(nt, 0);
  m->tb_rounds.assign((size_t)nb * (kTBMaxRounds + 1), 0);
  std::vector<int> adj;
  std::vector<int32_t> order;
  uint64_t seed = 0x9e3779b97f4a7c15ull;
  for (int b = 0; b < nb; ++b) {
    const int t0 = m->tb_t0[b], t1 = m->tb_t0[b + 1], n = t1 - t0;
    adj.assign(3 * (size_t)n, -1);
    for (int t = t0; t < t1; ++t)
      for (int a = 0; a < 3; ++a) {
        const int e = m->tedge[3 * (size_t)t + a];
        if (e < 0) continue;
        const int o = E[6 * (size_t)e + 2] == t ? E[6 * (size_t)e + 3] : E[6 * (size_t)e + 2];
        if (o >= t0 && o < t1) adj[3 * (size_t)(t - t0) + a] = o - t0;
      }
    order.assign(n, 0);
    if (!block_rounds(adj, n, kTBRound, kTBMaxRounds, order.data(),
                      &m->tb_rounds[(size_t)b * (kTBMaxRounds + 1)], seed))
      return;
    for (int i = 0; i < n; ++i) m->tb_order[t0 + i] = t0 + order[i];
  }
  m->tb_tiles.clear();
  for (int I = 0; I < nb; ++I)
    for (int J = I; J < nb; ++J)
      m->tb_tiles.push_back((int32_t)(((uint32_t)I << 16) | (uint32_t)J));
  m->tb_ok = true;
}

template <class T>
static bool take(Arena &A, T **dst, size_t n) {
  T *p = nullptr;
  if (!A.bottom(&p, n)) return false;
  if (dst) *dst = p;
  return true;
}

// Every device array of a mesh, carved from its workspace in a fixed order
// (d == nullptr: count only).
static bool carve_mesh(const mf_mesh *m, Arena &A, mf_mesh *d) {
  const size_t npair = std::max<size_t>(m->touch_q.size(), 1);
  const size_t nt = (size_t)m->nt;
#define MF_TAKE(field, n) take(A, d ? &d->field : nullptr, (n))
  return MF_TAKE(d_tri, m->tri.size()) && MF_TAKE(d_tedge, m->tedge.size()) &&
         MF_TAKE(d_edges, m->edges.size()) && MF_TAKE(d_tsign, m->tsign.size()) &&
         MF_TAKE(d_touch_off, m->touch_off.size()) && MF_TAKE(d_touch_q, m->touch_q.size()) &&
         MF_TAKE(d_touch_rev, m->touch_rev.size()) && MF_TAKE(d_touch_p, m->touch_p.size()) &&
         MF_TAKE(d_touch_u, m->touch_u.size()) &&
         MF_TAKE(d_blk_off, m->blk_off.size()) && MF_TAKE(d_blk_tri, m->blk_tri.size()) &&
         MF_TAKE(d_blk_pos, m->blk_pos.size()) && MF_TAKE(d_tiles, m->tiles.size()) &&
         MF_TAKE(d_blk_e0, m->blk_e0.size()) && MF_TAKE(d_blk_rt, m->blk_rt.size()) &&
         MF_TAKE(d_blk_ord, m->blk_ord.size()) && MF_TAKE(d_blk_rounds, m->blk_rounds.size()) &&
         MF_TAKE(d_elen, (size_t)m->ne) && MF_TAKE(d_sing1, 18 * npair) &&
         MF_TAKE(d_sing, 18 * npair) && MF_TAKE(d_scratch, 16) && MF_TAKE(d_status, 4) &&
         MF_TAKE(d_qp64, 3 * kMaxQ * nt) && MF_TAKE(d_brad, 4 * nt) &&
         MF_TAKE(d_rec, (size_t)kRecFloats * nt) && MF_TAKE(d_sph, 4 * (size_t)range_runs(m->nt)) &&
         MF_TAKE(d_tb_t0, m->tb_t0.size()) && MF_TAKE(d_tb_e0, m->tb_e0.size()) &&
         MF_TAKE(d_tb_nbe, m->tb_nbe.size()) && MF_TAKE(d_tb_be_off, m->tb_be_off.size()) &&
         MF_TAKE(d_tb_be_cut, m->tb_be_cut.size()) && MF_TAKE(d_tb_pos, m->tb_pos.size()) &&
         MF_TAKE(d_tb_order, m->tb_order.size()) && MF_TAKE(d_tb_rounds, m->tb_rounds.size()) &&
         MF_TAKE(d_tb_tiles, m->tb_tiles.size()) && MF_TAKE(d_cut_idx, m->cut_idx.size()) &&
         MF_TAKE(d_cut_edge, m->cut_edge.size()) &&
         MF_TAKE(d_side, m->tb_ok ? 2 * (size_t)m->n_cut * ((size_t)m->ne + m->n_cut) : 0);
#undef MF_TAKE
}

template <class T>
static int upload(T *dst, const std::vector<T> &src, hipStream_t s) {
  if (!src.empty())
    MF_HIP(hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s));
  return MF_OK;
}

static bool g_timing = false;

static void free_mesh(mf_mesh *m) {
  if (!m) return;
  for (hipEvent_t &e : m->ev)
    if (e) (void)hipEventDestroy(e);
  delete m;  // the device workspace belongs to the caller
}

// Calls that run on the GPU need the caller's workspace bound to the mesh.
static int ensure_device(mf_mesh *m) {
  if (m->ws) return MF_OK;
  set_error("mesh has no device workspace (mf_mesh_workspace_bytes, mf_mesh_set_workspace)");
  return MF_EINVAL;
}

}  // namespace mf

struct mf_near {
  mf_mesh *mesh = nullptr;
  double r_near = 0.0;
  std::vector<int64_t> row_ptr;  // E + 1
  std::vector<int32_t> col;      // nnz, sorted per row
  std::vector<int32_t> tiles;    // (I << 16) | J, I <= J, tiles holding a near pair
  std::vector<int32_t> toff;     // tiles + 1
  std::vector<int32_t> ent;      // 4 ints per entry
  int32_t *d_tiles = nullptr, *d_toff = nullptr, *d_ent = nullptr;
};

struct mf_batch {
  mf::Rule r;
  int part = 0;
  std::vector<mf_mesh *> mesh;
  std::vector<const double *> V;
  std::vector<double> k;
  std::vector<float *> sing;  // per-item touching-pair blocks (in the workspace)
  std::vector<float *> side;  // per-item cut-edge side buffers (in the workspace)
  mf::FillLaunch *launch = nullptr;
  int threads = 0;             // workgroup size picked by the tuner
  int shape = 0;               // tile shape picked by the tuner (0 edge, 1 triangle blocks)
  float tune_ms[mf::kBatchChoices] = {};
};

using namespace mf;

extern "C" {

const char *mf_last_error(void) { return g_err.c_str(); }

int mf_mesh_create(int32_t n_vertices, int32_t n_triangles, const int32_t *triangles,
                   mf_mesh **out) {
  if (!out || !triangles || n_vertices <= 0 || n_triangles <= 0)
    return fail(MF_EINVAL, "mf_mesh_create: bad argument");
  *out = nullptr;
  mf_mesh *m = new (std::nothrow) mf_mesh;
  if (!m) return fail(MF_ENOMEM, "mf_mesh_create: out of host memory");
  m->nv = n_vertices;
  m->nt = n_triangles;
  m->tri.assign(triangles, triangles + 3 * (size_t)n_triangles);
  int rc = build_topology(m);
  if (rc) {
    free_mesh(m);
    return rc;
  }
  build_touching(m);
  build_blocks(m);
  build_tb_plan(m);
  if (m->nblk > 65535) {
    free_mesh(m);
    return fail(MF_EINVAL, "mf_mesh_create: too many RWG edges for the tile plan");
  }
  if (m->max_blk_tris > kMaxBlockTris) {
    free_mesh(m);
    return fail(MF_EMESH, "internal: edge block needs too many triangles");
  }
  *out = m;
  return MF_OK;
}

void mf_mesh_destroy(mf_mesh *mesh) { free_mesh(mesh); }

int mf_mesh_n_edges(const mf_mesh *m, int32_t *n) {
  if (!m || !n) return fail(MF_EINVAL, "mf_mesh_n_edges: bad argument");
  *n = m->ne;
  return MF_OK;
}

int mf_mesh_edges(const mf_mesh *m, int32_t *edges) {
  if (!m || !edges) return fail(MF_EINVAL, "mf_mesh_edges: bad argument");
  std::memcpy(edges, m->edges.data(), m->edges.size() * sizeof(int32_t));
  return MF_OK;
}

int mf_mesh_n_touching(const mf_mesh *m, int64_t *n) {
  if (!m || !n) return fail(MF_EINVAL, "mf_mesh_n_touching: bad argument");
  *n = (int64_t)m->touch_q.size();
  return MF_OK;
}

int mf_mesh_plan(const mf_mesh *m, int32_t *n_blocks, int64_t *n_tiles,
                 int32_t *max_block_triangles) {
  if (!m || !n_blocks || !n_tiles || !max_block_triangles)
    return fail(MF_EINVAL, "mf_mesh_plan: bad argument");
  *n_blocks = m->nblk;
  *n_tiles = (int64_t)m->tiles.size();
  *max_block_triangles = m->max_blk_tris;
  return MF_OK;
}

int mf_mesh_tb_plan(const mf_mesh *m, int32_t *n_blocks, int64_t *n_tiles, int32_t *n_cut,
                    int32_t *max_rounds) {
  if (!m || !n_blocks || !n_tiles || !n_cut || !max_rounds)
    return fail(MF_EINVAL, "mf_mesh_tb_plan: bad argument");
  *n_blocks = m->tb_ok ? m->tb_nblk : 0;
  *n_tiles = m->tb_ok ? (int64_t)m->tb_tiles.size() : 0;
  *n_cut = m->tb_ok ? m->n_cut : 0;
  int mr = 0;
  for (int b = 0; m->tb_ok && b < m->tb_nblk; ++b) {
    const int32_t *rs = &m->tb_rounds[(size_t)b * (kTBMaxRounds + 1)];
    int r = 0;
    while (r < kTBMaxRounds && rs[r + 1] > rs[r]) ++r;
    mr = std::max(mr, r);
  }
  *max_rounds = mr;
  return MF_OK;
}

int mf_mesh_workspace_bytes(const mf_mesh *m, size_t *bytes) {
  if (!m || !bytes) return fail(MF_EINVAL, "mf_mesh_workspace_bytes: bad argument");
  Arena A = Arena::counter();
  carve_mesh(m, A, nullptr);
  *bytes = A.lo;
  return MF_OK;
}

int mf_mesh_set_workspace(mf_mesh *m, void *ws, size_t bytes, hipStream_t s) {
  if (!m || !ws) return fail(MF_EINVAL, "mf_mesh_set_workspace: bad argument");
  if ((uintptr_t)ws & 255) return fail(MF_EINVAL, "mf_mesh_set_workspace: workspace not 256-byte aligned");
  Arena A(ws, bytes);
  mf_mesh view;  // carve into a scratch handle first: a short workspace leaves m unchanged
  if (!carve_mesh(m, A, &view)) return fail(MF_EINVAL, "mf_mesh_set_workspace: workspace too small");
  carve_mesh(m, A = Arena(ws, bytes), m);
  m->ws = ws;
  m->ws_bytes = bytes;
  int rc;
  if ((rc = upload(m->d_tri, m->tri, s)) || (rc = upload(m->d_tedge, m->tedge, s)) ||
      (rc = upload(m->d_edges, m->edges, s)) || (rc = upload(m->d_tsign, m->tsign, s)) ||
      (rc = upload(m->d_touch_off, m->touch_off, s)) ||
      (rc = upload(m->d_touch_q, m->touch_q, s)) ||
      (rc = upload(m->d_touch_rev, m->touch_rev, s)) ||
      (rc = upload(m->d_touch_p, m->touch_p, s)) || (rc = upload(m->d_touch_u, m->touch_u, s)) ||
      (rc = upload(m->d_blk_off, m->blk_off, s)) ||
      (rc = upload(m->d_blk_tri, m->blk_tri, s)) || (rc = upload(m->d_blk_pos, m->blk_pos, s)) ||
      (rc = upload(m->d_tiles, m->tiles, s)) || (rc = upload(m->d_blk_e0, m->blk_e0, s)) ||
      (rc = upload(m->d_blk_rt, m->blk_rt, s)) || (rc = upload(m->d_blk_ord, m->blk_ord, s)) ||
      (rc = upload(m->d_blk_rounds, m->blk_rounds, s)) || (rc = upload(m->d_tb_t0, m->tb_t0, s)) ||
      (rc = upload(m->d_tb_e0, m->tb_e0, s)) || (rc = upload(m->d_tb_nbe, m->tb_nbe, s)) ||
      (rc = upload(m->d_tb_be_off, m->tb_be_off, s)) ||
      (rc = upload(m->d_tb_be_cut, m->tb_be_cut, s)) || (rc = upload(m->d_tb_pos, m->tb_pos, s)) ||
      (rc = upload(m->d_tb_order, m->tb_order, s)) ||
      (rc = upload(m->d_tb_rounds, m->tb_rounds, s)) ||
      (rc = upload(m->d_tb_tiles, m->tb_tiles, s)) || (rc = upload(m->d_cut_idx, m->cut_idx, s)) ||
      (rc = upload(m->d_cut_edge, m->cut_edge, s))) {
    m->ws = nullptr;
    return rc;
  }
  hipError_t e = hipMemsetAsync(m->d_status, 0, sizeof(int) * 4, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    m->ws = nullptr;
    return hip_fail(e, "mf_mesh_set_workspace");
  }
  return MF_OK;
}

int mf_r_range(mf_mesh *m, const double *V, int quad_order, double *rmin, double *rmax,
               hipStream_t s) {
  Rule r;
  if (!m || !V || !rmin || !rmax || !make_rule(quad_order, &r))
    return fail(MF_EINVAL, "mf_r_range: bad argument (quad_order must be 3, 6 or 7)");
  int rc = ensure_device(m);
  if (rc) return rc;
  if ((rc = launch_geometry(m, V, r, s))) return rc;
  return launch_r_range(m, V, r, rmin, rmax, s);
}

int mf_r_range_static(mf_mesh *m, const double *V, int quad_order, double *rmin, double *rmax,
                      hipStream_t s) {
  Rule r;
  if (!m || !V || !rmin || !rmax || !make_rule(quad_order, &r))
    return fail(MF_EINVAL, "mf_r_range_static: bad argument (quad_order must be 3, 6 or 7)");
  if (m->nt > max_static_range_triangles())
    return fail(MF_EINVAL, "mf_r_range_static: more triangles than the static scratch holds (" +
                               std::to_string(max_static_range_triangles()) + ")");
  int rc = ensure_device(m);
  if (rc) return rc;
  if ((rc = launch_geometry(m, V, r, s))) return rc;
  return launch_r_range_static(m, V, r, rmin, rmax, s);
}

static int check_table_args(const char *who, double k, double rmin, double rmax, double tol,
                            bool green) {
  const std::string w = who;
  if (!(k > 0.0) || !std::isfinite(k)) return fail(MF_EINVAL, w + ": k must be > 0");
  if (green && (!(rmin > 0.0) || !(rmax > rmin) || !std::isfinite(rmax)))
    return fail(MF_EINVAL, w + ": need 0 < r_min < r_max");
  if (!green && (!(rmax > 0.0) || !std::isfinite(rmax)))
    return fail(MF_EINVAL, w + ": need r_max > 0");
  if (!(tol >= 1e-12 && tol <= 1e-1)) return fail(MF_EINVAL, w + ": tol must lie in [1e-12, 1e-1]");
  return MF_OK;
}

int mf_tables_workspace_bytes(double k, double rmin, double rmax, double tol, size_t *bytes) {
  if (!bytes) return fail(MF_EINVAL, "mf_tables_workspace_bytes: bytes is NULL");
  int rc = check_table_args("mf_tables_workspace_bytes", k, rmin, rmax, tol, true);
  if (rc) return rc;
  *bytes = tables_workspace_bytes(k, rmin, rmax, tol, true);
  return MF_OK;
}

int mf_exp_table_workspace_bytes(double k, double rmax, double tol, size_t *bytes) {
  if (!bytes) return fail(MF_EINVAL, "mf_exp_table_workspace_bytes: bytes is NULL");
  int rc = check_table_args("mf_exp_table_workspace_bytes", k, 0.0, rmax, tol, false);
  if (rc) return rc;
  *bytes = tables_workspace_bytes(k, 0.0, rmax, tol, false);
  return MF_OK;
}

static int build_into(const char *who, double k, double rmin, double rmax, double tol, bool green,
                      void *ws, size_t bytes, mf_tables **out, hipStream_t s) {
  if (!out) return fail(MF_EINVAL, std::string(who) + ": out is NULL");
  *out = nullptr;
  int rc = check_table_args(who, k, rmin, rmax, tol, green);
  if (rc) return rc;
  if (!ws || ((uintptr_t)ws & 255))
    return fail(MF_EINVAL, std::string(who) + ": workspace NULL or not 256-byte aligned");
  mf_tables *t = new (std::nothrow) mf_tables;
  if (!t) return fail(MF_ENOMEM, std::string(who) + ": out of host memory");
  t->k = k;
  t->rmin = rmin;
  t->rmax = rmax;
  t->tol = tol;
  t->arena = Arena(ws, bytes);
  rc = build_tables_device(t, tol, s, green);
  if (rc) {
    mf_tables_destroy(t);
    return rc;
  }
  *out = t;
  return MF_OK;
}

int mf_build_tables(double k, double rmin, double rmax, double tol, void *ws, size_t bytes,
                    mf_tables **out, hipStream_t s) {
  return build_into("mf_build_tables", k, rmin, rmax, tol, true, ws, bytes, out, s);
}

int mf_build_exp_table(double k, double rmax, double tol, void *ws, size_t bytes, mf_tables **out,
                       hipStream_t s) {
  return build_into("mf_build_exp_table", k, 0.0, rmax, tol, false, ws, bytes, out, s);
}

void mf_tables_destroy(mf_tables *t) {
  if (!t) return;
  release_tables(t);
  delete t;
}

int mf_tables_info(const mf_tables *t, int32_t *n_exp, int32_t *n_green, int32_t *m_exp,
                   int32_t *m_green, double *t_exp, double *t_green, double *err_exp,
                   double *err_green) {
  if (!t) return fail(MF_EINVAL, "mf_tables_info: tables is NULL");
  if (n_exp) *n_exp = t->e.n;
  if (n_green) *n_green = t->g.n;
  if (m_exp) *m_exp = t->e.m;
  if (m_green) *m_green = t->g.m;
  if (t_exp) *t_exp = t->e.t;
  if (t_green) *t_green = t->g.t;
  if (err_exp) *err_exp = t->e.err;
  if (err_green) *err_green = t->g.err;
  return MF_OK;
}

int mf_tables_get(const mf_tables *t, int which, double *r, double *values, int32_t *hash,
                  hipStream_t s) {
  if (!t || (which != 0 && which != 1)) return fail(MF_EINVAL, "mf_tables_get: bad argument");
  const mf_tables::One &o = which == 0 ? t->e : t->g;
  if (r) MF_HIP(hipMemcpyAsync(r, o.r, sizeof(double) * o.n, hipMemcpyDeviceToHost, s));
  if (values)
    MF_HIP(hipMemcpyAsync(values, o.f, sizeof(double) * 2 * o.n, hipMemcpyDeviceToHost, s));
  if (hash) MF_HIP(hipMemcpyAsync(hash, o.hash, sizeof(int32_t) * o.m, hipMemcpyDeviceToHost, s));
  MF_HIP(hipStreamSynchronize(s));
  return MF_OK;
}

int mf_tables_eval(const mf_tables *t, int which, int64_t n, const double *r, double *out,
                   hipStream_t s) {
  if (!t || (which != 0 && which != 1) || n < 0 || (n > 0 && (!r || !out)))
    return fail(MF_EINVAL, "mf_tables_eval: bad argument");
  if ((which == 0 ? t->e.n : t->g.n) == 0)
    return fail(MF_EINVAL, "mf_tables_eval: this table was not built");
  if (n == 0) return MF_OK;
  return launch_table_eval(t, which, n, r, out, s);
}

int mf_fill_Z(mf_mesh *m, const double *V, double k, int quad_order, int mode,
              const mf_tables *tab, void *Z, int z_dtype, int64_t ldz, hipStream_t s) {
  Rule r;
  if (!m || !V || !Z) return fail(MF_EINVAL, "mf_fill_Z: NULL argument");
  if (!make_rule(quad_order, &r)) return fail(MF_EINVAL, "mf_fill_Z: quad_order must be 3, 6 or 7");
  if (!(k > 0.0) || !std::isfinite(k)) return fail(MF_EINVAL, "mf_fill_Z: k must be > 0");
  const int base = mode & 0xf, part = mode & (MF_PART_A | MF_PART_PHI);
  if ((base != MF_MODE_TABLE && base != MF_MODE_DIRECT) || (mode & ~0x3f) ||
      part == (MF_PART_A | MF_PART_PHI))
    return fail(MF_EINVAL, "mf_fill_Z: unknown mode");
  if (base == MF_MODE_TABLE && (!tab || tab->g.n == 0))
    return fail(MF_EINVAL, "mf_fill_Z: table mode needs a Green table");
  if (base == MF_MODE_TABLE && std::fabs(tab->k - k) > 1e-12 * k)
    return fail(MF_EINVAL, "mf_fill_Z: tables were built for another k");
  if (z_dtype != MF_C64 && z_dtype != MF_C128) return fail(MF_EINVAL, "mf_fill_Z: unknown z_dtype");
  if (ldz < m->ne) return fail(MF_EINVAL, "mf_fill_Z: ldz < number of edges");
  int rc = ensure_device(m);
  if (rc) return rc;
  const bool timed = g_timing;
  if (timed && !m->ev[0])
    for (hipEvent_t &e : m->ev) MF_HIP(hipEventCreate(&e));
  if (timed) MF_HIP(hipEventRecord(m->ev[0], s));
  if ((rc = launch_geometry(m, V, r, s))) return rc;
  if (timed) MF_HIP(hipEventRecord(m->ev[1], s));
  if ((rc = launch_singular(m, V, r, k, part, s))) return rc;
  if (timed) MF_HIP(hipEventRecord(m->ev[2], s));
  m->timing_now = timed;
  m->split = false;
  rc = launch_fill(m, r, k, mode, tab, Z, z_dtype, ldz, s);
  m->timing_now = false;
  if (rc) return rc;
  if (timed) MF_HIP(hipEventRecord(m->ev[3], s));
  m->timed = timed;
  return MF_OK;
}

int mf_fill_mfie(mf_mesh *m, const double *V, double k, int quad_order, int mode,
                 const mf_tables *tab, void *Z, int z_dtype, int64_t ldz, hipStream_t s) {
  Rule r;
  if (!m || !V || !Z) return fail(MF_EINVAL, "mf_fill_mfie: NULL argument");
  if (!make_rule(quad_order, &r))
    return fail(MF_EINVAL, "mf_fill_mfie: quad_order must be 3, 6 or 7");
  if (!(k > 0.0) || !std::isfinite(k)) return fail(MF_EINVAL, "mf_fill_mfie: k must be > 0");
  if (mode != MF_MODE_TABLE && mode != MF_MODE_DIRECT)
    return fail(MF_EINVAL, "mf_fill_mfie: unknown mode");
  if (mode == MF_MODE_TABLE && (!tab || tab->g.n == 0))
    return fail(MF_EINVAL, "mf_fill_mfie: table mode needs a Green table");
  if (mode == MF_MODE_TABLE && std::fabs(tab->k - k) > 1e-12 * k)
    return fail(MF_EINVAL, "mf_fill_mfie: tables were built for another k");
  if (z_dtype != MF_C64 && z_dtype != MF_C128)
    return fail(MF_EINVAL, "mf_fill_mfie: unknown z_dtype");
  if (ldz < m->ne) return fail(MF_EINVAL, "mf_fill_mfie: ldz < number of edges");
  int rc = ensure_device(m);
  if (rc) return rc;
  const bool timed = g_timing;
  if (timed && !m->ev[0])
    for (hipEvent_t &e : m->ev) MF_HIP(hipEventCreate(&e));
  if (timed) MF_HIP(hipEventRecord(m->ev[0], s));
  if ((rc = launch_geometry(m, V, r, s))) return rc;
  if (timed) MF_HIP(hipEventRecord(m->ev[1], s));
  if ((rc = launch_singular_mfie(m, V, r, k, s))) return rc;
  if (timed) MF_HIP(hipEventRecord(m->ev[2], s));
  if ((rc = launch_fill(m, r, k, mode | kModeMfie, tab, Z, z_dtype, ldz, s))) return rc;
  if (timed) MF_HIP(hipEventRecord(m->ev[3], s));
  m->timed = timed;
  return MF_OK;
}

int mf_angular_rmax(mf_mesh *m, const double *V, int quad_order, double *rmax, hipStream_t s) {
  Rule r;
  if (!m || !V || !rmax) return fail(MF_EINVAL, "mf_angular_rmax: NULL argument");
  if (!make_rule(quad_order, &r))
    return fail(MF_EINVAL, "mf_angular_rmax: quad_order must be 3, 6 or 7");
  int rc = ensure_device(m);
  if (rc) return rc;
  if ((rc = launch_geometry(m, V, r, s))) return rc;
  return launch_range_angular(m, V, r, rmax, s);
}

int mf_fill_angular(mf_mesh *m, const double *V, double k, int quad_order, int n_edge, int mode,
                    const mf_tables *tab, void *Z, int z_dtype, int64_t ldz, hipStream_t s) {
  Rule r;
  if (!m || !V || !Z) return fail(MF_EINVAL, "mf_fill_angular: NULL argument");
  if (!make_rule(quad_order, &r))
    return fail(MF_EINVAL, "mf_fill_angular: quad_order must be 3, 6 or 7");
  if (n_edge != 4 && n_edge != 6 && n_edge != 8)
    return fail(MF_EINVAL, "mf_fill_angular: points per edge must be 4, 6 or 8");
  if (!(k > 0.0) || !std::isfinite(k)) return fail(MF_EINVAL, "mf_fill_angular: k must be > 0");
  if (mode != MF_MODE_TABLE && mode != MF_MODE_DIRECT)
    return fail(MF_EINVAL, "mf_fill_angular: unknown mode");
  if (mode == MF_MODE_TABLE &&
      (!tab || tab->e.n < 2 || !tab->e.look64 || tab->rmin != 0.0 ||
       std::fabs(tab->k - k) > 1e-12 * k))
    return fail(MF_EINVAL,
                "mf_fill_angular: table mode needs an Exp table from r = 0 built for this k");
  if (z_dtype != MF_C64 && z_dtype != MF_C128)
    return fail(MF_EINVAL, "mf_fill_angular: unknown z_dtype");
  if (ldz < m->ne) return fail(MF_EINVAL, "mf_fill_angular: ldz < number of edges");
  int rc = ensure_device(m);
  if (rc) return rc;
  const bool timed = g_timing;
  if (timed && !m->ev[0])
    for (hipEvent_t &e : m->ev) MF_HIP(hipEventCreate(&e));
  if (timed) MF_HIP(hipEventRecord(m->ev[0], s));
  if ((rc = launch_geometry(m, V, r, s))) return rc;
  if (timed) {
    MF_HIP(hipEventRecord(m->ev[1], s));
    MF_HIP(hipEventRecord(m->ev[2], s));  // no separate touching-pair phase
  }
  if ((rc = launch_fill_angular(m, V, r, k, n_edge, mode, tab, Z, z_dtype, ldz, s))) return rc;
  if (timed) MF_HIP(hipEventRecord(m->ev[3], s));
  m->timed = timed;
  return MF_OK;
}

// The batch's device arrays: per item its touching-pair blocks, then the
// item list of the launch (d == nullptr: count only).
// The batch's workspace: per item its touching-pair blocks and, when every
// mesh has a triangle-block plan, a cut-edge side buffer (each item fills
// its own, so items that share a mesh can run in one launch), then the item
// list.
static bool carve_batch(int n, mf_mesh *const *meshes, Arena &A, std::vector<float *> *sing,
                        std::vector<float *> *side, void **items) {
  bool tb = n > 1;
  for (int i = 0; i < n; ++i) tb = tb && meshes[i]->tb_ok;
  for (int i = 0; i < n; ++i) {
    float *p = nullptr;
    if (!A.bottom(&p, 18 * std::max<size_t>(meshes[i]->touch_q.size(), 1))) return false;
    if (sing) (*sing)[i] = p;
    float *q = nullptr;
    if (tb && !A.bottom(&q, 2 * (size_t)meshes[i]->n_cut *
                                ((size_t)meshes[i]->ne + meshes[i]->n_cut)))
      return false;
    if (side) (*side)[i] = q;
  }
  char *it = nullptr;
  if (!A.bottom(&it, fill_items_bytes(n))) return false;
  if (items) *items = it;
  return true;
}

int mf_batch_workspace_bytes(int32_t n, mf_mesh *const *meshes, size_t *bytes) {
  if (n < 1 || !meshes || !bytes) return fail(MF_EINVAL, "mf_batch_workspace_bytes: bad argument");
  for (int i = 0; i < n; ++i)
    if (!meshes[i]) return fail(MF_EINVAL, "mf_batch_workspace_bytes: NULL mesh");
  Arena A = Arena::counter();
  carve_batch(n, meshes, A, nullptr, nullptr, nullptr);
  *bytes = A.lo;
  return MF_OK;
}

int mf_batch_create(int32_t n, mf_mesh *const *meshes, const double *const *V, const double *k,
                    const mf_tables *const *tab, int quad_order, int mode, void *const *Z,
                    int z_dtype, const int64_t *ldz, void *ws, size_t ws_bytes, mf_batch **out) {
  Rule r;
  if (n < 1 || !meshes || !V || !k || !Z || !ldz || !out || !ws)
    return fail(MF_EINVAL, "mf_batch_create: bad argument");
  if ((uintptr_t)ws & 255) return fail(MF_EINVAL, "mf_batch_create: workspace not 256-byte aligned");
  *out = nullptr;
  if (!make_rule(quad_order, &r))
    return fail(MF_EINVAL, "mf_batch_create: quad_order must be 3, 6 or 7");
  const int base = mode & 0xf, part = mode & (MF_PART_A | MF_PART_PHI);
  if ((base != MF_MODE_TABLE && base != MF_MODE_DIRECT) || (mode & ~0x3f) ||
      part == (MF_PART_A | MF_PART_PHI))
    return fail(MF_EINVAL, "mf_batch_create: unknown mode");
  if (z_dtype != MF_C64 && z_dtype != MF_C128)
    return fail(MF_EINVAL, "mf_batch_create: unknown z_dtype");
  if (base == MF_MODE_TABLE && !tab)
    return fail(MF_EINVAL, "mf_batch_create: table mode needs tables");
  for (int i = 0; i < n; ++i) {
    const std::string at = "mf_batch_create: item " + std::to_string(i) + ": ";
    if (!meshes[i] || !V[i] || !Z[i]) return fail(MF_EINVAL, at + "NULL argument");
    if (!(k[i] > 0.0) || !std::isfinite(k[i])) return fail(MF_EINVAL, at + "k must be > 0");
    if (base == MF_MODE_TABLE &&
        (!tab[i] || tab[i]->g.n == 0 || std::fabs(tab[i]->k - k[i]) > 1e-12 * k[i]))
      return fail(MF_EINVAL, at + "tables missing, without a Green table or built for another k");
    if (ldz[i] < meshes[i]->ne) return fail(MF_EINVAL, at + "ldz < number of edges");
    for (int j = 0; j < i; ++j)
      if (meshes[j] == meshes[i] && V[j] != V[i])
        return fail(MF_EINVAL, at + "a mesh shared by two items needs one vertex pointer");
  }
  mf_batch *b = new (std::nothrow) mf_batch;
  if (!b) return fail(MF_ENOMEM, "mf_batch_create: out of host memory");
  b->r = r;
  b->part = part;
  b->mesh.assign(meshes, meshes + n);
  b->V.assign(V, V + n);
  b->k.assign(k, k + n);
  int rc = MF_OK;
  for (int i = 0; i < n && !rc; ++i) rc = ensure_device(meshes[i]);
  b->sing.assign(n, nullptr);
  b->side.assign(n, nullptr);
  void *items = nullptr;
  Arena A(ws, ws_bytes);
  if (!rc && !carve_batch(n, meshes, A, &b->sing, &b->side, &items))
    rc = fail(MF_EINVAL, "mf_batch_create: workspace too small (mf_batch_workspace_bytes)");
  if (!rc) {
    std::vector<const float *> sing(b->sing.begin(), b->sing.end());
    const bool sides = n > 1 && b->side[0] != nullptr;
    rc = fill_launch_create(n, meshes, k, tab, r, mode, Z, z_dtype, ldz, sing.data(), items,
                            &b->launch, sides ? b->side.data() : nullptr);
  }
  // tile-shape tuning on the real inputs: geometry and touching blocks first,
  // then the launch variants (writing the outputs); all on the null stream
  if (!rc) {
    *out = b;
    rc = mf_batch_fill(b, nullptr);
    if (!rc) rc = fill_launch_autotune(b->launch, nullptr, b->tune_ms, &b->threads, &b->shape);
    if (!rc) {
      hipError_t e = hipStreamSynchronize(nullptr);
      if (e != hipSuccess) rc = hip_fail(e, "mf_batch_create: tuning");
    }
  }
  if (rc) {
    *out = nullptr;
    mf_batch_destroy(b);
    return rc;
  }
  *out = b;
  return MF_OK;
}

int mf_batch_info(const mf_batch *b, int32_t *threads, int32_t *tile_shape, float *tune_ms5) {
  if (!b) return fail(MF_EINVAL, "mf_batch_info: batch is NULL");
  if (threads) *threads = b->threads;
  if (tile_shape) *tile_shape = b->shape;
  if (tune_ms5)
    for (int i = 0; i < kBatchChoices; ++i) tune_ms5[i] = b->tune_ms[i];
  return MF_OK;
}

int mf_batch_set_choice(mf_batch *b, int32_t choice) {
  if (!b) return fail(MF_EINVAL, "mf_batch_set_choice: batch is NULL");
  const int rc = fill_launch_set_choice(b->launch, choice);
  if (rc) return rc;
  b->shape = choice >= 3 ? 1 : 0;
  b->threads = choice == 0 ? 512 : choice == 1 ? 768 : choice == 4 ? 512 : 1024;
  return MF_OK;
}

int mf_batch_fill(mf_batch *b, hipStream_t s) {
  if (!b) return fail(MF_EINVAL, "mf_batch_fill: batch is NULL");
  const int n = (int)b->mesh.size();
  int rc;
  for (int i = 0; i < n; ++i) {
    bool seen = false;
    for (int j = 0; j < i; ++j) seen |= b->mesh[j] == b->mesh[i];
    if (!seen && (rc = launch_geometry(b->mesh[i], b->V[i], b->r, s))) return rc;
  }
  for (int i = 0; i < n; ++i)
    if ((rc = launch_singular(b->mesh[i], b->V[i], b->r, b->k[i], b->part, s, b->sing[i])))
      return rc;
  return fill_launch_run(b->launch, s);
}

void mf_batch_destroy(mf_batch *b) {
  if (!b) return;
  fill_launch_destroy(b->launch);
  delete b;  // the device workspace belongs to the caller
}

int mf_near_create(mf_mesh *m, const double *V, double r_near, mf_near **out) {
  if (!m || !V || !out || !(r_near > 0.0) || !std::isfinite(r_near))
    return fail(MF_EINVAL, "mf_near_create: bad argument");
  *out = nullptr;
  const int ne = m->ne;
  // edge midpoints, bucketed in a grid of cells of side r_near
  std::vector<double> mid(3 * (size_t)ne);
  double lo[3] = {1e300, 1e300, 1e300};
  for (int e = 0; e < ne; ++e)
    for (int c = 0; c < 3; ++c) {
      const int32_t *E = &m->edges[6 * (size_t)e];
      mid[3 * e + c] = 0.5 * (V[3 * (size_t)E[0] + c] + V[3 * (size_t)E[1] + c]);
      lo[c] = std::min(lo[c], mid[3 * e + c]);
    }
  std::map<std::array<int64_t, 3>, std::vector<int32_t>> cells;
  auto cell_of = [&](int e) {
    std::array<int64_t, 3> key;
    for (int c = 0; c < 3; ++c) key[c] = (int64_t)std::floor((mid[3 * e + c] - lo[c]) / r_near);
    return key;
  };
  for (int e = 0; e < ne; ++e) cells[cell_of(e)].push_back(e);
  mf_near *nf = new (std::nothrow) mf_near;
  if (!nf) return fail(MF_ENOMEM, "mf_near_create: out of host memory");
  nf->mesh = m;
  nf->r_near = r_near;
  nf->row_ptr.assign(ne + 1, 0);
  const double r2 = r_near * r_near;
  std::vector<int32_t> row;
  for (int e = 0; e < ne; ++e) {
    row.clear();
    const std::array<int64_t, 3> k0 = cell_of(e);
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dz = -1; dz <= 1; ++dz) {
          auto it = cells.find({k0[0] + dx, k0[1] + dy, k0[2] + dz});
          if (it == cells.end()) continue;
          for (int32_t f : it->second) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
              const double d = mid[3 * e + c] - mid[3 * (size_t)f + c];
              d2 += d * d;
            }
            if (d2 <= r2) row.push_back(f);
          }
        }
    std::sort(row.begin(), row.end());
    nf->col.insert(nf->col.end(), row.begin(), row.end());
    nf->row_ptr[e + 1] = (int64_t)nf->col.size();
  }
  if (nf->col.size() > (size_t)INT32_MAX) {
    mf_near_destroy(nf);
    return fail(MF_EINVAL, "mf_near_create: more than 2^31 near pairs");
  }
  // block of every edge, then the tiles (I <= J) that hold a near pair
  std::vector<int32_t> blk(ne);
  for (int b = 0; b < m->nblk; ++b)
    for (int e = m->blk_e0[b]; e < m->blk_e0[b + 1]; ++e) blk[e] = b;
  std::map<int32_t, std::vector<std::array<int32_t, 4>>> per_tile;
  auto pos = [&](int r, int c) -> int32_t {
    const auto b = nf->col.begin() + nf->row_ptr[r], e = nf->col.begin() + nf->row_ptr[r + 1];
    return (int32_t)(std::lower_bound(b, e, c) - nf->col.begin());
  };
  for (int e = 0; e < ne; ++e)
    for (int64_t s = nf->row_ptr[e]; s < nf->row_ptr[e + 1]; ++s) {
      const int f = nf->col[s];
      const int I = blk[e], J = blk[f];
      if (I > J) continue;  // taken as the mirror of (f, e)
      const int r = e - m->blk_e0[I], c = f - m->blk_e0[J];
      // on a diagonal tile both orders are computed, so no mirror write
      per_tile[(int32_t)(((uint32_t)I << 16) | (uint32_t)J)].push_back({(r << 8) | c, (int32_t)s, I == J ? -1 : pos(f, e), 0});
    }
  nf->toff.push_back(0);
  for (auto &kv : per_tile) {
    nf->tiles.push_back(kv.first);
    for (auto &en : kv.second) nf->ent.insert(nf->ent.end(), en.begin(), en.end());
    nf->toff.push_back((int32_t)(nf->ent.size() / 4));
  }
  *out = nf;  // device copies follow at the first fill
  return MF_OK;
}

int mf_near_info(const mf_near *nf, int64_t *nnz, int64_t *n_tiles) {
  if (!nf || !nnz || !n_tiles) return fail(MF_EINVAL, "mf_near_info: bad argument");
  *nnz = (int64_t)nf->col.size();
  *n_tiles = (int64_t)nf->tiles.size();
  return MF_OK;
}

int mf_near_pattern(const mf_near *nf, int64_t *row_ptr, int32_t *col) {
  if (!nf || !row_ptr || !col) return fail(MF_EINVAL, "mf_near_pattern: bad argument");
  std::memcpy(row_ptr, nf->row_ptr.data(), sizeof(int64_t) * nf->row_ptr.size());
  std::memcpy(col, nf->col.data(), sizeof(int32_t) * nf->col.size());
  return MF_OK;
}

static bool carve_near(const mf_near *nf, Arena &A, mf_near *d) {
  int32_t *a = nullptr, *b = nullptr, *c = nullptr;
  if (!A.bottom(&a, nf->tiles.size()) || !A.bottom(&b, nf->toff.size()) ||
      !A.bottom(&c, nf->ent.size()))
    return false;
  if (d) {
    d->d_tiles = a;
    d->d_toff = b;
    d->d_ent = c;
  }
  return true;
}

int mf_near_workspace_bytes(const mf_near *nf, size_t *bytes) {
  if (!nf || !bytes) return fail(MF_EINVAL, "mf_near_workspace_bytes: bad argument");
  Arena A = Arena::counter();
  carve_near(nf, A, nullptr);
  *bytes = A.lo;
  return MF_OK;
}

int mf_near_set_workspace(mf_near *nf, void *ws, size_t bytes, hipStream_t s) {
  if (!nf || !ws) return fail(MF_EINVAL, "mf_near_set_workspace: bad argument");
  if ((uintptr_t)ws & 255) return fail(MF_EINVAL, "mf_near_set_workspace: workspace not 256-byte aligned");
  Arena A(ws, bytes);
  mf_near view;
  if (!carve_near(nf, A, &view)) return fail(MF_EINVAL, "mf_near_set_workspace: workspace too small");
  nf->d_tiles = view.d_tiles;
  nf->d_toff = view.d_toff;
  nf->d_ent = view.d_ent;
  int rc;
  if ((rc = upload(nf->d_tiles, nf->tiles, s)) || (rc = upload(nf->d_toff, nf->toff, s)) ||
      (rc = upload(nf->d_ent, nf->ent, s))) {
    nf->d_ent = nullptr;
    return rc;
  }
  MF_HIP(hipStreamSynchronize(s));
  return MF_OK;
}

int mf_fill_near(mf_mesh *m, mf_near *nf, const double *V, double k, int quad_order,
                 int mode, const mf_tables *tab, void *values, int z_dtype, hipStream_t s) {
  Rule r;
  if (!m || !nf || !V || !values || nf->mesh != m)
    return fail(MF_EINVAL, "mf_fill_near: bad argument (the pattern belongs to another mesh?)");
  if (!make_rule(quad_order, &r)) return fail(MF_EINVAL, "mf_fill_near: quad_order must be 3, 6 or 7");
  if (!(k > 0.0) || !std::isfinite(k)) return fail(MF_EINVAL, "mf_fill_near: k must be > 0");
  if (mode != MF_MODE_TABLE && mode != MF_MODE_DIRECT)
    return fail(MF_EINVAL, "mf_fill_near: unknown mode");
  if (mode == MF_MODE_TABLE && (!tab || tab->g.n == 0 || std::fabs(tab->k - k) > 1e-12 * k))
    return fail(MF_EINVAL, "mf_fill_near: tables missing, without a Green table or built for another k");
  if (z_dtype != MF_C64 && z_dtype != MF_C128) return fail(MF_EINVAL, "mf_fill_near: unknown z_dtype");
  int rc = ensure_device(m);
  if (rc) return rc;
  if (!nf->d_ent)
    return fail(MF_EINVAL, "mf_fill_near: pattern has no device workspace (mf_near_set_workspace)");
  if ((rc = launch_geometry(m, V, r, s))) return rc;
  if ((rc = launch_singular(m, V, r, k, 0, s))) return rc;
  if (nf->tiles.empty()) return MF_OK;
  return launch_fill_near(m, r, k, mode, tab, nf->d_tiles, (int)nf->tiles.size(), nf->d_toff,
                          reinterpret_cast<const int4 *>(nf->d_ent), values, z_dtype, s);
}

void mf_near_destroy(mf_near *nf) { delete nf; }  // the device workspace belongs to the caller

int mf_rhs_planewave(mf_mesh *m, const double *V, double k, int quad_order, const double *khat,
                     const double *E0, void *out, int z_dtype, hipStream_t s) {
  Rule r;
  if (!m || !V || !khat || !E0 || !out) return fail(MF_EINVAL, "mf_rhs_planewave: NULL argument");
  if (!make_rule(quad_order, &r))
    return fail(MF_EINVAL, "mf_rhs_planewave: quad_order must be 3, 6 or 7");
  if (!(k >= 0.0) || !std::isfinite(k)) return fail(MF_EINVAL, "mf_rhs_planewave: k must be >= 0");
  if (z_dtype != MF_C64 && z_dtype != MF_C128)
    return fail(MF_EINVAL, "mf_rhs_planewave: unknown z_dtype");
  const double kn = std::sqrt(khat[0] * khat[0] + khat[1] * khat[1] + khat[2] * khat[2]);
  if (!(std::fabs(kn - 1.0) < 1e-9)) return fail(MF_EINVAL, "mf_rhs_planewave: khat must be a unit vector");
  int rc = ensure_device(m);
  if (rc) return rc;
  return launch_rhs(m, V, r, k, khat, E0, out, z_dtype, s);
}

int mf_rhs_planewave_mfie(mf_mesh *m, const double *V, double k, int quad_order,
                          const double *khat, const double *E0, void *out, int z_dtype,
                          hipStream_t s) {
  Rule r;
  if (!m || !V || !khat || !E0 || !out)
    return fail(MF_EINVAL, "mf_rhs_planewave_mfie: NULL argument");
  if (!make_rule(quad_order, &r))
    return fail(MF_EINVAL, "mf_rhs_planewave_mfie: quad_order must be 3, 6 or 7");
  if (!(k >= 0.0) || !std::isfinite(k))
    return fail(MF_EINVAL, "mf_rhs_planewave_mfie: k must be >= 0");
  if (z_dtype != MF_C64 && z_dtype != MF_C128)
    return fail(MF_EINVAL, "mf_rhs_planewave_mfie: unknown z_dtype");
  const double kn = std::sqrt(khat[0] * khat[0] + khat[1] * khat[1] + khat[2] * khat[2]);
  if (!(std::fabs(kn - 1.0) < 1e-9))
    return fail(MF_EINVAL, "mf_rhs_planewave_mfie: khat must be a unit vector");
  int rc = ensure_device(m);
  if (rc) return rc;
  return launch_rhs(m, V, r, k, khat, E0, out, z_dtype, s, true);
}

int mf_far_field(mf_mesh *m, const double *V, double k, int quad_order, const void *I,
                 int z_dtype, int32_t n_dirs, const double *dirs, double e0_norm, double *F,
                 double *sigma, hipStream_t s) {
  Rule r;
  if (!m || !V || !I || !dirs || !F || n_dirs < 0)
    return fail(MF_EINVAL, "mf_far_field: bad argument");
  if (!make_rule(quad_order, &r)) return fail(MF_EINVAL, "mf_far_field: quad_order must be 3, 6 or 7");
  if (!(k > 0.0) || !std::isfinite(k)) return fail(MF_EINVAL, "mf_far_field: k must be > 0");
  if (z_dtype != MF_C64 && z_dtype != MF_C128) return fail(MF_EINVAL, "mf_far_field: unknown z_dtype");
  if (sigma && !(e0_norm > 0.0)) return fail(MF_EINVAL, "mf_far_field: e0_norm must be > 0");
  int rc = ensure_device(m);
  if (rc) return rc;
  if (n_dirs == 0) return MF_OK;
  return launch_far_field(m, V, r, k, I, z_dtype, n_dirs, dirs, e0_norm * e0_norm, F, sigma, s);
}

void mf_set_timing(int on) { g_timing = on != 0; }

int mf_mesh_timings(mf_mesh *m, float *ms3) {
  if (!m || !ms3 || !m->timed) return fail(MF_EINVAL, "mf_mesh_timings: no timed fill");
  MF_HIP(hipEventSynchronize(m->ev[3]));
  for (int i = 0; i < 3; ++i) MF_HIP(hipEventElapsedTime(&ms3[i], m->ev[i], m->ev[i + 1]));
  return MF_OK;
}

int mf_mesh_fill_timings(mf_mesh *m, float *ms2) {
  if (!m || !ms2 || !m->timed) return fail(MF_EINVAL, "mf_mesh_fill_timings: no timed fill");
  MF_HIP(hipEventSynchronize(m->ev[3]));
  if (!m->split) {
    MF_HIP(hipEventElapsedTime(&ms2[0], m->ev[2], m->ev[3]));
    ms2[1] = 0.0f;
    return MF_OK;
  }
  MF_HIP(hipEventElapsedTime(&ms2[0], m->ev[2], m->ev[4]));
  MF_HIP(hipEventElapsedTime(&ms2[1], m->ev[4], m->ev[3]));
  return MF_OK;
}

int mf_fill_Z_backward(mf_mesh *m, const double *V, double k, int quad_order, int mode,
                       const mf_tables *tab, const void *W, int z_dtype, int64_t ldz, double *dV,
                       double *dk, hipStream_t s) {
  Rule r;
  if (!m || !V || !W || !dV || !dk) return fail(MF_EINVAL, "mf_fill_Z_backward: NULL argument");
  if (!make_rule(quad_order, &r))
    return fail(MF_EINVAL, "mf_fill_Z_backward: quad_order must be 3, 6 or 7");
  if (!(k > 0.0) || !std::isfinite(k)) return fail(MF_EINVAL, "mf_fill_Z_backward: k must be > 0");
  if (mode != MF_MODE_TABLE && mode != MF_MODE_DIRECT)
    return fail(MF_EINVAL, "mf_fill_Z_backward: unknown mode");
  if (mode == MF_MODE_TABLE && (!tab || tab->g.n == 0))
    return fail(MF_EINVAL, "mf_fill_Z_backward: table mode needs the Green and Exp tables");
  if (z_dtype != MF_C64 && z_dtype != MF_C128)
    return fail(MF_EINVAL, "mf_fill_Z_backward: unknown z_dtype");
  if (ldz < m->ne) return fail(MF_EINVAL, "mf_fill_Z_backward: ldz < number of edges");
  int rc = ensure_device(m);
  if (rc) return rc;
  if ((rc = launch_geometry(m, V, r, s))) return rc;
  return launch_backward(m, V, r, k, mode, tab, W, z_dtype, ldz, dV, dk, s);
}

int mf_sync_status(mf_mesh *m, hipStream_t s) {
  if (!m) return fail(MF_EINVAL, "mf_sync_status: mesh is NULL");
  if (!m->d_status) return MF_OK;
  MF_HIP(hipStreamSynchronize(s));
  int st[4];
  MF_HIP(hipMemcpy(st, m->d_status, sizeof(st), hipMemcpyDeviceToHost));
  if (st[0] != 0) {
    MF_HIP(hipMemset(m->d_status, 0, sizeof(int) * 4));
    return fail(MF_ERANGE, "a regular-pair distance fell outside the table range");
  }
  return MF_OK;
}

}  // extern "C"
