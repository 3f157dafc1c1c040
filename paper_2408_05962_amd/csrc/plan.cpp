// Host side of the executor: registration, race check, hierarchical
// factorization with striping, channel split, dependency DAG, ordering,
// tiling, byte accounting and the host-memory schedule checker.
//
// Method: HiCCL (arXiv 2408.05962), Sec. 3 (primitives, steps, fences) and
// Sec. 4 (tree factorization Sec. 4.2, striping Sec. 4.3, factorization
// order Sec. 4.4, pipelining Sec. 4.5). The readings used where the paper is
// silent are stated next to the code that applies them.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <numeric>
#include <queue>
#include <random>
#include <tuple>
#include <set>
#include <unordered_map>

#include "hiccl_impl.hpp"

namespace hiccl {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

// ---------------------------------------------------------------- hierarchy
// Ranks per depth-k group: B[0] = P, B[L] = 1 (Sec. 4.2: consecutive ranks
// fill the innermost groups, the first factor is the highest level).
static std::vector<int> group_sizes(const std::vector<int>& h, int P) {
  std::vector<int> B(h.size() + 1);
  B[0] = P;
  for (size_t k = 0; k < h.size(); ++k) B[k + 1] = B[k] / h[k];
  return B;
}

// Depth (1 = highest level) at which ranks a and b first fall into
// different groups; 0 when a == b.
int hier_depth(int a, int b, const std::vector<int>& h) {
  if (a == b) return 0;
  int P = 1;
  for (int f : h) P *= f;
  int size = P;
  for (size_t k = 0; k < h.size(); ++k) {
    size /= h[k];
    if (a / size != b / size) return int(k) + 1;
  }
  return int(h.size());
}

// Contiguous pieces of n elements with boundaries on multiples of `align`;
// whole units spread evenly (earlier pieces take the extra unit), the last
// piece also takes the sub-unit remainder.
static std::vector<std::pair<uint64_t, uint64_t>> split_range(uint64_t n, int parts, uint64_t align) {
  std::vector<std::pair<uint64_t, uint64_t>> out;
  uint64_t units = n / align, rem = n % align, off = 0;
  for (int t = 0; t < parts; ++t) {
    uint64_t u = units / parts + (uint64_t(t) < units % parts ? 1 : 0);
    uint64_t len = u * align + (t == parts - 1 ? rem : 0);
    out.push_back({off, len});
    off += len;
  }
  return out;
}

static uint64_t round_up(uint64_t x, uint64_t a) { return (x + a - 1) / a * a; }

uint64_t tile_elems_for(size_t tile_bytes, int dtype) {
  uint64_t al = align_elems(dtype);
  uint64_t e = tile_bytes / elem_size(dtype);
  e = e / al * al;
  return e < al ? al : e;
}

// -------------------------------------------------------------- factorizer
namespace {

struct RNode {                    // reduction tree node or leaf
  int host = 0;
  int leaf = -1;                  // >= 0: a contributing rank, no node
  std::vector<RNode> kids;
};

struct Factorizer {
  const Comm& c;
  const Prim& p;
  int dt;
  std::vector<int> B;
  int L;
  uint64_t& ws_top;
  std::vector<Op>& ops;

  int kr = 0;                     // depth whose groups are the ring's conceptual nodes (0: no ring)

  Factorizer(const Comm& c_, const Prim& p_, uint64_t& ws, std::vector<Op>& out)
      : c(c_), p(p_), dt(c_.dtype), B(group_sizes(c_.hier, c_.P)), L(int(c_.hier.size())), ws_top(ws), ops(out) {
    if (c.ring > 1)
      for (int k = 1; k <= L; ++k)
        if (B[k] == c.P / c.ring) kr = k;
  }

  // First ranks of the conceptual nodes the ring visits after the one of
  // rank `r`, in ring order (the next node, the one after, ...), skipping
  // nodes that hold no leaf (Sec. 4.4).
  std::vector<int> ring_chain(int r, const std::vector<int>& leaves) const {
    std::vector<int> out;
    const int size = B[kr], mine = r / size;
    for (int ci = 1; ci < c.ring; ++ci) {
      int lo = ((mine + ci) % c.ring) * size;
      for (int x : leaves)
        if (x >= lo && x < lo + size) {
          out.push_back(lo);
          break;
        }
    }
    return out;
  }

  static std::vector<int> in_range(const std::vector<int>& v, int lo, int hi, int skip_a = -1, int skip_b = -1) {
    std::vector<int> o;
    for (int x : v)
      if (x >= lo && x < hi && x != skip_a && x != skip_b) o.push_back(x);
    return o;
  }

  Loc user(const hiccl_buf_t& b, uint64_t off) const {
    Loc l;
    l.space = 0;
    l.addr = uint64_t(reinterpret_cast<uintptr_t>(b.data));
    l.scales = uint64_t(reinterpret_cast<uintptr_t>(b.scales));
    return l.at(off, dt);
  }

  Loc ws(uint64_t n) {
    Loc l;
    l.space = 1;
    l.addr = ws_top;
    ws_top += round_up(n * elem_size(dt), 256);
    if (dt == HICCL_FP8_E4M3) {
      l.scales = ws_top;
      ws_top += round_up((n / kFp8Block) * sizeof(float), 256);
    }
    return l;
  }

  void copy(const Loc& s, int sr, const Loc& d, int dr, bool dws, uint64_t n, uint64_t off, int stripe,
            bool whole = false, int ring_step = 0) {
    Op o;
    o.ring_step = ring_step;
    o.kind = kCopy;
    o.src = {s};
    o.src_rank = {sr};
    o.dst = d;
    o.dst_rank = dr;
    o.dst_ws = dws;
    o.count = n;
    o.offset = off;
    o.stripe = stripe;
    o.whole = whole;
    ops.push_back(std::move(o));
  }

  // Stripe owners (reading: the root's smallest enclosing group whose size
  // is >= s and divisible by s; owner t sits at the root's offset plus
  // t*size/s modulo the group size). Empty when the primitive is not
  // striped: s == 1, or every leaf already inside that group.
  std::vector<int> owners(const std::vector<int>& leaves) const {
    int s = c.stripe;
    if (s <= 1) return {};
    for (int k = L; k >= kr; --k) {
      int size = B[k];
      if (size >= s && size % s == 0) {
        int lo = p.root / size * size;
        bool outside = false;
        for (int x : leaves)
          if (x < lo || x >= lo + size) outside = true;
        if (!outside) return {};
        std::vector<int> o(s);
        for (int t = 0; t < s; ++t) o[t] = lo + ((p.root - lo) + t * (size / s)) % size;
        return o;
      }
    }
    return {};
  }

  // Tree multicast of Sec. 4.2: `src` holds the branch at `sl`; it sends
  // one copy into each sibling group holding leaves (to the staging rank:
  // the same-offset rank if it is a leaf, else the group's lowest leaf),
  // which then multicasts inside its group; the own group is handled by
  // `src` itself one level down.
  void mcast(int src, const Loc& sl, const std::vector<int>& lv, int lo, int k, uint64_t off, uint64_t n,
             int stripe) {
    if (k > L || lv.empty()) return;
    int sub = B[k];
    int mine = (src - lo) / sub;
    for (int ci = 0; ci < c.hier[k - 1]; ++ci) {
      int clo = lo + ci * sub;
      std::vector<int> cl;
      for (int x : lv)
        if (x >= clo && x < clo + sub) cl.push_back(x);
      if (ci == mine) {
        std::vector<int> rest;
        for (int x : cl)
          if (x != src) rest.push_back(x);
        mcast(src, sl, rest, clo, k + 1, off, n, stripe);
      } else if (!cl.empty()) {
        int same = clo + (src - lo) % sub;
        int stg = std::find(cl.begin(), cl.end(), same) != cl.end() ? same : cl.front();
        Loc d = user(p.recv[stg], off);
        copy(sl, src, d, stg, false, n, off, stripe);
        std::vector<int> rest;
        for (int x : cl)
          if (x != stg) rest.push_back(x);
        mcast(stg, d, rest, clo, k + 1, off, n, stripe);
      }
    }
  }

  void multicast() {
    std::vector<int> leaves = p.leaves;
    std::sort(leaves.begin(), leaves.end());
    int r = p.root;
    Loc rs = user(p.send[r], 0);
    bool root_leaf = std::binary_search(leaves.begin(), leaves.end(), r);
    if (root_leaf && p.send[r].data != p.recv[r].data)
      copy(rs, r, user(p.recv[r], 0), r, false, p.count, 0, 0, true);
    std::vector<int> others;
    for (int x : leaves)
      if (x != r) others.push_back(x);
    std::vector<int> own = owners(leaves);
    if (kr > 0) {
      // ring + tree (Sec. 4.4): striping, then each stripe runs along a rail through the
      // conceptual nodes, then a tree inside every node
      std::vector<std::pair<uint64_t, uint64_t>> pieces =
          own.empty() ? std::vector<std::pair<uint64_t, uint64_t>>{{0, p.count}}
                      : split_range(p.count, int(own.size()), align_elems(dt));
      if (own.empty()) own = {r};
      const int size = B[kr], lo0 = r / size * size;
      std::vector<int> chain = ring_chain(r, leaves);
      for (size_t t = 0; t < own.size(); ++t) {
        uint64_t off = pieces[t].first, len = pieces[t].second;
        if (len == 0) continue;
        int o = own[t];
        int stripe = own.size() > 1 ? int(t) : 0;
        Loc ol;
        if (o == r) {
          ol = rs.at(off, dt);
        } else {
          bool oleaf = std::binary_search(leaves.begin(), leaves.end(), o);
          ol = oleaf ? user(p.recv[o], off) : ws(len);
          copy(rs.at(off, dt), r, ol, o, !oleaf, len, off, stripe);
        }
        mcast(o, ol, in_range(leaves, lo0, lo0 + size, o, r), lo0, kr + 1, off, len, stripe);
        int prev = o;
        Loc pl = ol;
        for (size_t ci = 0; ci < chain.size(); ++ci) {
          int dst = chain[ci] + (o - lo0);
          bool dleaf = std::binary_search(leaves.begin(), leaves.end(), dst);
          Loc dl = dleaf ? user(p.recv[dst], off) : ws(len);
          copy(pl, prev, dl, dst, !dleaf, len, off, stripe, false, int(ci) + 1);
          mcast(dst, dl, in_range(leaves, chain[ci], chain[ci] + size, dst), chain[ci], kr + 1, off, len, stripe);
          prev = dst;
          pl = dl;
        }
      }
      return;
    }
    if (own.empty()) {
      mcast(r, rs, others, 0, 1, 0, p.count, 0);
      return;
    }
    // striping (Sec. 4.3): scatter the stripes to their owners, then one
    // multicast per stripe from its owner; the root already holds every
    // stripe, so the branches do not send back to it
    auto pieces = split_range(p.count, int(own.size()), align_elems(dt));
    for (size_t t = 0; t < own.size(); ++t) {
      uint64_t off = pieces[t].first, len = pieces[t].second;
      if (len == 0) continue;
      int o = own[t];
      Loc ol;
      if (o == r) {
        ol = rs.at(off, dt);
      } else {
        bool oleaf = std::binary_search(leaves.begin(), leaves.end(), o);
        ol = oleaf ? user(p.recv[o], off) : ws(len);
        copy(rs.at(off, dt), r, ol, o, !oleaf, len, off, int(t));
      }
      std::vector<int> lv;
      for (int x : leaves)
        if (x != o && x != r) lv.push_back(x);
      mcast(o, ol, lv, 0, 1, off, len, int(t));
    }
  }

  // Reduction tree rooted at `root` (the mirror of the multicast): a group
  // with several contributing subgroups forms one node hosted by the root
  // if it lies inside, else by the same-offset rank if it contributes,
  // else by the lowest contributing rank; a group with one contributing
  // subgroup forms no node.
  bool rtree(const std::vector<int>& lv, int root, int lo, int k, RNode& out) const {
    int size = B[k - 1];
    bool any = false;
    for (int x : lv)
      if (x >= lo && x < lo + size) any = true;
    if (!any) return false;
    if (size == 1) {
      out.leaf = lo;
      out.host = lo;
      return true;
    }
    int sub = B[k];
    std::vector<RNode> kids;
    for (int ci = 0; ci < c.hier[k - 1]; ++ci) {
      RNode ch;
      if (rtree(lv, root, lo + ci * sub, k + 1, ch)) kids.push_back(std::move(ch));
    }
    if (kids.size() == 1) {
      out = std::move(kids[0]);
      return true;
    }
    int host;
    if (root >= lo && root < lo + size) {
      host = root;
    } else {
      int same = lo + root % size;
      host = std::binary_search(lv.begin(), lv.end(), same) ? same : -1;
      if (host < 0)
        for (int x : lv)
          if (x >= lo && x < lo + size) {
            host = x;
            break;
          }
    }
    out.leaf = -1;
    out.host = host;
    out.kids = std::move(kids);
    return true;
  }

  // Emit a node's operands first, then the node. Operands are combined in
  // ascending child-group order. Returns the location of the node value.
  Loc emit_node(const RNode& nd, uint64_t off, uint64_t n, int stripe, const Loc* final_dst, bool final_ws,
                const Loc* extra = nullptr, int extra_rank = -1, int ring_step = 0) {
    Op o;
    o.kind = kReduce;
    o.ring_step = ring_step;
    for (const RNode& ch : nd.kids) {
      if (ch.leaf >= 0) {
        o.src.push_back(user(p.send[ch.leaf], off));
      } else {
        o.src.push_back(emit_node(ch, off, n, stripe, nullptr, true));
      }
      o.src_rank.push_back(ch.host);
    }
    if (extra) {          // the partial arriving from the next node of the ring, last
      o.src.push_back(*extra);
      o.src_rank.push_back(extra_rank);
    }
    o.dst = final_dst ? *final_dst : ws(n);
    o.dst_ws = final_dst ? final_ws : true;
    o.dst_rank = nd.host;
    o.count = n;
    o.offset = off;
    o.stripe = stripe;
    Loc d = o.dst;
    ops.push_back(std::move(o));
    return d;
  }

  // One node of a ring reduction: reduce the node's leaves by its inner
  // tree rooted at `holder`; the top operation also takes `inc` (the partial
  // from the next node), last. Writes `dst` if given, else workspace.
  Loc ring_node(const std::vector<int>& leaves, int lo, int holder, const Loc* inc, int inc_rank, uint64_t off,
                uint64_t n, int stripe, int step, const Loc* dst, bool dst_ws) {
    const int size = B[kr];
    std::vector<int> lv = in_range(leaves, lo, lo + size);
    Loc out = dst ? *dst : ws(n);
    if (lv.empty()) {              // nothing to add here: only the arriving partial moves on
      if (inc && !(inc->space == out.space && inc->addr == out.addr))
        copy(*inc, inc_rank, out, holder, dst ? dst_ws : true, n, off, stripe, false, step);
      return out;
    }
    RNode tree;
    rtree(lv, holder, lo, kr + 1, tree);
    if (tree.leaf >= 0) {
      Loc s = user(p.send[tree.leaf], off);
      if (inc) {
        Op o;
        o.kind = kReduce;
        o.ring_step = step;
        o.src = {s, *inc};
        o.src_rank = {tree.leaf, inc_rank};
        o.dst = out;
        o.dst_ws = dst ? dst_ws : true;
        o.dst_rank = holder;
        o.count = n;
        o.offset = off;
        o.stripe = stripe;
        ops.push_back(std::move(o));
      } else if (!(s.space == out.space && s.addr == out.addr)) {
        copy(s, tree.leaf, out, holder, dst ? dst_ws : true, n, off, stripe);
      }
      return out;
    }
    return emit_node(tree, off, n, stripe, &out, dst ? dst_ws : true, inc, inc_rank, step);
  }

  // Ring reduction (mirror of the ring multicast): the farthest node of the
  // chain starts, each node adds its own leaves and forwards, the node of
  // `o` finishes into `fin`.
  void ring_reduce(const std::vector<int>& leaves, int o, uint64_t off, uint64_t n, int stripe, const Loc& fin,
                   bool fin_ws) {
    const int size = B[kr], lo0 = o / size * size;
    std::vector<int> chain = ring_chain(o, leaves);
    Loc inc;
    int inc_rank = -1;
    bool have = false;
    for (int ci = int(chain.size()) - 1; ci >= 0; --ci) {
      int holder = chain[ci] + (o - lo0);
      inc = ring_node(leaves, chain[ci], holder, have ? &inc : nullptr, inc_rank, off, n, stripe, ci + 2, nullptr,
                      true);
      inc_rank = holder;
      have = true;
    }
    ring_node(leaves, lo0, o, have ? &inc : nullptr, inc_rank, off, n, stripe, 1, &fin, fin_ws);
  }

  void reduction() {
    std::vector<int> leaves = p.leaves;
    std::sort(leaves.begin(), leaves.end());
    int j = p.root;
    std::vector<int> own = owners(leaves);
    std::vector<std::pair<uint64_t, uint64_t>> pieces;
    if (own.empty()) {
      pieces = {{0, p.count}};
      own = {j};
    } else {
      pieces = split_range(p.count, int(own.size()), align_elems(dt));
    }
    for (size_t t = 0; t < own.size(); ++t) {
      uint64_t off = pieces[t].first, len = pieces[t].second;
      if (len == 0) continue;
      int o = own[t];
      int stripe = own.size() > 1 ? int(t) : 0;
      Loc fin = (o == j) ? user(p.recv[j], off) : ws(len);
      bool fin_ws = (o != j);
      if (kr > 0) {
        ring_reduce(leaves, o, off, len, stripe, fin, fin_ws);
        if (o != j) copy(fin, o, user(p.recv[j], off), j, false, len, off, stripe);
        continue;
      }
      RNode tree;
      rtree(leaves, o, 0, 1, tree);
      if (tree.leaf >= 0) {
        // one contributing rank: point-to-point, the unary operation omitted
        Loc s = user(p.send[tree.leaf], off);
        if (!(s.space == fin.space && s.addr == fin.addr)) copy(s, tree.leaf, fin, o, fin_ws, len, off, stripe);
      } else {
        emit_node(tree, off, len, stripe, &fin, fin_ws);
      }
      // striped reduction (mirror of Sec. 4.3): the owner's result goes to the root
      if (o != j) copy(fin, o, user(p.recv[j], off), j, false, len, off, stripe);
    }
  }
};

// ------------------------------------------------- dependency interval index
struct Range {
  int space;
  uint64_t lo, hi;
  bool write;
};

static void task_ranges(const Task& t, std::vector<Range>& out) {
  out.clear();
  size_t es = elem_size(t.dtype);
  uint64_t nb = t.count * es;
  bool fp8 = t.dtype == HICCL_FP8_E4M3;
  uint64_t nsb = fp8 ? (t.count / kFp8Block) * sizeof(float) : 0;
  for (const Loc& s : t.src) {
    out.push_back({s.space, s.addr, s.addr + nb, false});
    if (fp8) out.push_back({s.space, s.scales, s.scales + nsb, false});
  }
  out.push_back({t.dst.space, t.dst.addr, t.dst.addr + nb, true});
  if (fp8) out.push_back({t.dst.space, t.dst.scales, t.dst.scales + nsb, true});
}

struct IntervalIndex {
  struct Entry {
    uint64_t hi;
    int task;
    bool write;
  };
  std::multimap<uint64_t, Entry> by_lo[2];
  uint64_t maxlen[2] = {0, 0};

  void insert(const Range& r, int task) {
    if (r.hi <= r.lo) return;
    by_lo[r.space].insert({r.lo, Entry{r.hi, task, r.write}});
    maxlen[r.space] = std::max(maxlen[r.space], r.hi - r.lo);
  }
  template <class F>
  void conflicts(const Range& r, F&& f) const {
    if (r.hi <= r.lo) return;
    const auto& m = by_lo[r.space];
    uint64_t from = r.lo > maxlen[r.space] ? r.lo - maxlen[r.space] : 0;
    for (auto it = m.lower_bound(from); it != m.end() && it->first < r.hi; ++it) {
      const Entry& e = it->second;
      if (e.hi > r.lo && (e.write || r.write)) f(e.task);
    }
  }
};

}  // namespace

// Build tasks of one communicator into `out` (logical order, no tiling).
static int factorize_all(const Comm& c, std::vector<Task>& out, uint64_t& ws_top) {
  for (size_t pi = 0; pi < c.prims.size(); ++pi) {
    const Prim& p = c.prims[pi];
    if (p.count == 0 || p.leaves.empty()) continue;
    std::vector<Op> ops;
    Factorizer f(c, p, ws_top, ops);
    if (p.kind == 0)
      f.multicast();
    else
      f.reduction();
    for (const Op& o : ops) {
      auto chans = split_range(o.count, c.pipe, align_elems(c.dtype));
      for (int ch = 0; ch < c.pipe; ++ch) {
        uint64_t off = chans[ch].first, len = chans[ch].second;
        if (len == 0) continue;
        Task t;
        t.kind = o.kind;
        t.op = p.op;
        t.dtype = c.dtype;
        for (const Loc& s : o.src) t.src.push_back(s.at(off, c.dtype));
        t.src_rank = o.src_rank;
        t.dst = o.dst.at(off, c.dtype);
        t.dst_rank = o.dst_rank;
        t.dst_ws = o.dst_ws;
        t.count = len;
        t.offset = o.offset + off;
        t.prim = int(pi);
        t.step = p.step;
        t.stripe = o.stripe;
        t.channel = ch;
        t.ring_step = o.ring_step;
        out.push_back(std::move(t));
      }
    }
  }
  return HICCL_SUCCESS;
}

// Dependencies: a task depends on every earlier task (in program order,
// which is topological) whose write overlaps its reads or writes, or
// whose reads overlap its write — on the same rank's memory. Across a
// fence this is exactly the fine-grain dependency of Sec. 3.3 (M_i waits
// only for R_i); inside a primitive it recovers the tree edges.
static void build_edges(std::vector<Task>& ts, uint64_t& nedges) {
  IntervalIndex idx;
  std::vector<Range> rs;
  nedges = 0;
  for (size_t i = 0; i < ts.size(); ++i) {
    task_ranges(ts[i], rs);
    std::vector<int> preds;
    for (const Range& r : rs) idx.conflicts(r, [&](int t) { preds.push_back(t); });
    std::sort(preds.begin(), preds.end());
    preds.erase(std::unique(preds.begin(), preds.end()), preds.end());
    ts[i].preds = preds;
    for (int pr : preds) ts[pr].succs.push_back(int(i));
    nedges += preds.size();
    for (const Range& r : rs) idx.insert(r, int(i));
  }
  for (size_t i = 0; i < ts.size(); ++i) {
    int s = 0;
    for (int pr : ts[i].preds) s = std::max(s, ts[pr].stage + 1);
    ts[i].stage = s;
  }
}

// One rank's share: the tasks whose output lies in rank r's memory, in
// program order. Edges from dropped tasks go (on separate GPUs they would be
// flags set by a peer) and the stages left are renumbered densely; every
// kept edge still runs from a lower stage to a higher one.
static void keep_share(std::vector<Task>& ts, int r, uint64_t& nedges) {
  std::vector<int> to(ts.size(), -1);
  std::vector<Task> kept;
  for (size_t i = 0; i < ts.size(); ++i)
    if (ts[i].dst_rank == r) {
      to[i] = int(kept.size());
      kept.push_back(std::move(ts[i]));
    }
  std::vector<int> stages;
  for (const Task& t : kept) stages.push_back(t.stage);
  std::sort(stages.begin(), stages.end());
  stages.erase(std::unique(stages.begin(), stages.end()), stages.end());
  auto remap = [&](std::vector<int>& v) {
    std::vector<int> o;
    for (int x : v)
      if (to[x] >= 0) o.push_back(to[x]);
    v.swap(o);
  };
  nedges = 0;
  for (Task& t : kept) {
    remap(t.preds);
    remap(t.succs);
    nedges += t.preds.size();
    t.stage = int(std::lower_bound(stages.begin(), stages.end(), t.stage) - stages.begin());
  }
  ts = std::move(kept);
}

void order_and_tile(Plan& p, int order, size_t tile_bytes) {
  std::vector<Task>& ts = p.tasks;
  size_t n = ts.size();
  std::vector<int> perm(n);
  std::iota(perm.begin(), perm.end(), 0);
  if (order == HICCL_ORDER_STAGE) {
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) { return ts[a].stage < ts[b].stage; });
  } else if (order == HICCL_ORDER_CRITICAL) {
    // within a stage, the task with the longest chain of successors first
    // (critical path first): a hop that feeds deeper subtrees starts
    // earlier, which is the schedule behind the tree and ring step counts of
    // Sec. 4.6. Edges run from lower to higher index, so one backward pass
    // computes every height.
    std::vector<int> height(n, 1);
    for (size_t i = n; i-- > 0;)
      for (int s : ts[i].succs) height[i] = std::max(height[i], height[s] + 1);
    std::stable_sort(perm.begin(), perm.end(), [&](int a, int b) {
      if (ts[a].stage != ts[b].stage) return ts[a].stage < ts[b].stage;
      return height[a] > height[b];
    });
  } else if (order == HICCL_ORDER_CHANNEL) {
    // Kahn's algorithm with the ready task of smallest (channel, stage, index) first: always a
    // topological order, even where splits of different sizes make channels depend across indices
    auto key = [&](int i) { return std::make_tuple(ts[i].channel, ts[i].stage, i); };
    auto cmp = [&](int a, int b) { return key(a) > key(b); };
    std::priority_queue<int, std::vector<int>, decltype(cmp)> ready(cmp);
    std::vector<int> indeg(n);
    for (size_t i = 0; i < n; ++i) {
      indeg[i] = int(ts[i].preds.size());
      if (!indeg[i]) ready.push(int(i));
    }
    perm.clear();
    while (!ready.empty()) {
      int i = ready.top();
      ready.pop();
      perm.push_back(i);
      for (int s : ts[i].succs)
        if (--indeg[s] == 0) ready.push(s);
    }
  }
  std::vector<int> inv(n);
  for (size_t i = 0; i < n; ++i) inv[perm[i]] = int(i);
  std::vector<Task> nt(n);
  for (size_t i = 0; i < n; ++i) {
    nt[i] = std::move(ts[perm[i]]);
    for (int& x : nt[i].preds) x = inv[x];
    for (int& x : nt[i].succs) x = inv[x];
    std::sort(nt[i].succs.begin(), nt[i].succs.end());
  }
  ts = std::move(nt);
  p.tile_task.clear();
  p.nstages = 0;
  for (size_t i = 0; i < n; ++i) {
    Task& t = ts[i];
    t.tile_elems = tile_elems_for(tile_bytes, t.dtype);
    t.ntiles = uint32_t((t.count + t.tile_elems - 1) / t.tile_elems);
    if (t.ntiles == 0) t.ntiles = 1;
    t.first_tile = uint32_t(p.tile_task.size());
    for (uint32_t k = 0; k < t.ntiles; ++k) p.tile_task.push_back(uint32_t(i));
    p.nstages = std::max(p.nstages, t.stage + 1);
  }
  p.stage_tile_begin.assign(p.nstages + 1, uint32_t(p.tile_task.size()));
  if (order == HICCL_ORDER_STAGE) {
    for (int i = int(n) - 1; i >= 0; --i) p.stage_tile_begin[ts[i].stage] = ts[i].first_tile;
    for (int s = p.nstages - 1; s >= 0; --s)
      p.stage_tile_begin[s] = std::min(p.stage_tile_begin[s], p.stage_tile_begin[s + 1]);
  }
  p.hbm_read = p.hbm_written = 0;
  for (const Task& t : ts) {
    uint64_t nb = t.count * elem_size(t.dtype);
    if (t.dtype == HICCL_FP8_E4M3) nb += (t.count / kFp8Block) * sizeof(float);
    p.hbm_read += nb * t.src.size();
    p.hbm_written += nb;
  }
}

int build_plan(Comm& c) {
  int P = 1;
  for (int f : c.hier) {
    if (f < 1) return fail(HICCL_ERR_INVALID_ARG, "hierarchy factors must be >= 1");
    P *= f;
  }
  if (P != c.P) return fail(HICCL_ERR_INVALID_ARG, "product of hierarchy factors must equal nranks");
  if (c.stripe < 1 || c.pipe < 1 || c.ring < 1)
    return fail(HICCL_ERR_INVALID_ARG, "stripe, ring and pipeline must be >= 1");
  if (c.stripe > 1) {
    auto B = group_sizes(c.hier, c.P);
    bool ok = false;
    for (int b : B)
      if (b >= c.stripe && b % c.stripe == 0) ok = true;
    if (!ok) return fail(HICCL_ERR_INVALID_ARG, "stripe factor divides no group of the hierarchy");
  }
  if (c.ring > 1) {
    auto B = group_sizes(c.hier, c.P);
    bool ok = c.P % c.ring == 0;
    int kr = -1;
    for (size_t k = 1; ok && k < B.size(); ++k)
      if (B[k] == c.P / c.ring) kr = int(k);
    if (!ok || kr < 0)
      return fail(HICCL_ERR_INVALID_ARG, "ring length must make nranks/ring a group size of the hierarchy");
    if (c.stripe > B[kr] || B[kr] % c.stripe)
      return fail(HICCL_ERR_INVALID_ARG, "with a ring, the stripe factor must divide the ring's node size");
  }
  Plan pl;
  uint64_t ws = 0;
  int rc = factorize_all(c, pl.tasks, ws);
  if (rc) return rc;
  build_edges(pl.tasks, pl.nedges);
  if (c.share >= 0) keep_share(pl.tasks, c.share, pl.nedges);
  // tile indices are 32-bit on the device
  uint64_t tiles = 0;
  for (const Task& t : pl.tasks) {
    const uint64_t te = tile_elems_for(c.exec.tile_bytes, t.dtype);
    tiles += std::max<uint64_t>(1, (t.count + te - 1) / te);
  }
  if (tiles >= (uint64_t(1) << 31))
    return fail(HICCL_ERR_INVALID_ARG, "the plan would need 2^31 or more tiles: use a larger tile size");
  int order = c.exec.mode == HICCL_EXEC_STAGED ? HICCL_ORDER_STAGE : c.exec.order;
  order_and_tile(pl, order, c.exec.tile_bytes);
  pl.ws_bytes = ws;
  c.plan = std::move(pl);
  return HICCL_SUCCESS;
}

// ------------------------------------------------------ host schedule check
namespace {

inline float bf16_to_f32(uint16_t b) {
  uint32_t u = uint32_t(b) << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}
inline uint16_t f32_to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return uint16_t(u >> 16);
}
inline float e4m3_to_f32(uint8_t c) {
  int e = (c >> 3) & 0xF, m = c & 7;
  float v = e == 0 ? std::ldexp(float(m), -9) : std::ldexp(float(8 + m), e - 10);
  return (c & 0x80) ? -v : v;
}
inline uint8_t f32_to_e4m3(float x) {
  uint8_t s = std::signbit(x) ? 0x80 : 0;
  float a = std::fabs(x);
  if (a >= 448.f) return s | 0x7E;
  if (a < 0.015625f) return s | uint8_t(std::nearbyint(a * 512.f));
  int ex;
  std::frexp(a, &ex);
  int e = ex - 1;
  int q = int(std::nearbyint(std::ldexp(a, 3 - e)));
  if (q == 16) {
    ++e;
    q = 8;
  }
  int code = ((e + 7) << 3) | (q - 8);
  if (code > 0x7E) code = 0x7E;
  return s | uint8_t(code);
}
inline float pow2_scale(float amax) {
  if (amax == 0.f) return 1.f;
  int ex;
  float f = std::frexp(amax, &ex);
  int e = f <= 0.875f ? ex - 9 : ex - 8;
  e = std::max(-126, std::min(127, e));
  return std::ldexp(1.f, e);
}

struct HostExec {
  const Plan& pl;
  uint8_t* ws;
  uint8_t* ptr(const Loc& l) const { return l.space == 0 ? reinterpret_cast<uint8_t*>(l.addr) : ws + l.addr; }
  float* sptr(const Loc& l) const {
    return reinterpret_cast<float*>(l.space == 0 ? reinterpret_cast<uint8_t*>(l.scales) : ws + l.scales);
  }

  void run(const Task& t) const {
    size_t es = elem_size(t.dtype);
    uint64_t n = t.count;
    if (t.kind == kCopy) {
      std::memmove(ptr(t.dst), ptr(t.src[0]), n * es);
      if (t.dtype == HICCL_FP8_E4M3)
        std::memmove(sptr(t.dst), sptr(t.src[0]), (n / kFp8Block) * sizeof(float));
      return;
    }
    size_t k = t.src.size();
    switch (t.dtype) {
      case HICCL_INT32: {
        std::vector<uint32_t> acc(n);
        std::memcpy(acc.data(), ptr(t.src[0]), n * 4);
        for (size_t j = 1; j < k; ++j) {
          const uint8_t* s = ptr(t.src[j]);
          for (uint64_t e = 0; e < n; ++e) {
            uint32_t v;
            std::memcpy(&v, s + e * 4, 4);
            int32_t a = int32_t(acc[e]), b = int32_t(v);
            acc[e] = t.op == HICCL_SUM ? acc[e] + v : uint32_t(t.op == HICCL_MAX ? std::max(a, b) : std::min(a, b));
          }
        }
        std::memcpy(ptr(t.dst), acc.data(), n * 4);
        break;
      }
      case HICCL_FLOAT32: {
        std::vector<float> acc(n);
        std::memcpy(acc.data(), ptr(t.src[0]), n * 4);
        for (size_t j = 1; j < k; ++j) {
          const uint8_t* s = ptr(t.src[j]);
          for (uint64_t e = 0; e < n; ++e) {
            float v;
            std::memcpy(&v, s + e * 4, 4);
            acc[e] = t.op == HICCL_SUM ? acc[e] + v : (t.op == HICCL_MAX ? std::fmax(acc[e], v) : std::fmin(acc[e], v));
          }
        }
        std::memcpy(ptr(t.dst), acc.data(), n * 4);
        break;
      }
      case HICCL_BFLOAT16: {
        std::vector<float> acc(n, 0.f);
        for (size_t j = 0; j < k; ++j) {
          const uint8_t* s = ptr(t.src[j]);
          for (uint64_t e = 0; e < n; ++e) {
            uint16_t v;
            std::memcpy(&v, s + e * 2, 2);
            acc[e] = j == 0 ? bf16_to_f32(v) : acc[e] + bf16_to_f32(v);
          }
        }
        uint8_t* d = ptr(t.dst);
        for (uint64_t e = 0; e < n; ++e) {
          uint16_t v = f32_to_bf16(acc[e]);
          std::memcpy(d + e * 2, &v, 2);
        }
        break;
      }
      case HICCL_FP8_E4M3: {
        std::vector<float> acc(n, 0.f);
        for (size_t j = 0; j < k; ++j) {
          const uint8_t* s = ptr(t.src[j]);
          const float* sc = sptr(t.src[j]);
          for (uint64_t e = 0; e < n; ++e) {
            float v = e4m3_to_f32(s[e]) * sc[e / kFp8Block];
            acc[e] = j == 0 ? v : acc[e] + v;
          }
        }
        uint8_t* d = ptr(t.dst);
        float* dsc = sptr(t.dst);
        for (uint64_t b = 0; b < n / kFp8Block; ++b) {
          float amax = 0.f;
          for (int e = 0; e < kFp8Block; ++e) amax = std::fmax(amax, std::fabs(acc[b * kFp8Block + e]));
          float sc = pow2_scale(amax);
          dsc[b] = sc;
          for (int e = 0; e < kFp8Block; ++e) d[b * kFp8Block + e] = f32_to_e4m3(acc[b * kFp8Block + e] / sc);
        }
        break;
      }
    }
  }
};

}  // namespace

static int validate_host(Comm& c, uint64_t seed, int norders) {
  const Plan& pl = c.plan;
  std::vector<uint8_t> ws(pl.ws_bytes + 256);
  // every caller range any task touches, snapshotted so each order starts from the same state
  std::vector<Range> rs, all;
  for (const Task& t : pl.tasks) {
    task_ranges(t, rs);
    for (const Range& r : rs)
      if (r.space == 0 && r.hi > r.lo) all.push_back(r);
  }
  std::sort(all.begin(), all.end(), [](const Range& a, const Range& b) { return a.lo < b.lo; });
  std::vector<std::pair<uint64_t, uint64_t>> merged;
  for (const Range& r : all) {
    if (!merged.empty() && r.lo <= merged.back().second)
      merged.back().second = std::max(merged.back().second, r.hi);
    else
      merged.push_back({r.lo, r.hi});
  }
  std::vector<std::vector<uint8_t>> snap, first;
  for (auto& m : merged) {
    const uint8_t* p = reinterpret_cast<const uint8_t*>(m.first);
    snap.emplace_back(p, p + (m.second - m.first));
  }
  std::mt19937_64 rng(seed);
  HostExec ex{pl, ws.data()};
  size_t n = pl.tasks.size();
  for (int o = 0; o < std::max(1, norders); ++o) {
    for (size_t i = 0; i < merged.size(); ++i)
      std::memcpy(reinterpret_cast<uint8_t*>(merged[i].first), snap[i].data(), snap[i].size());
    std::fill(ws.begin(), ws.end(), uint8_t(0xFF));   // NaN / -1 poison
    std::vector<int> indeg(n);
    std::vector<int> ready;
    for (size_t i = 0; i < n; ++i) {
      indeg[i] = int(pl.tasks[i].preds.size());
      if (!indeg[i]) ready.push_back(int(i));
    }
    size_t done = 0;
    while (!ready.empty()) {
      size_t pick = o == 0 ? 0 : size_t(rng() % ready.size());
      int t = ready[pick];
      ready[pick] = ready.back();
      ready.pop_back();
      ex.run(pl.tasks[t]);
      ++done;
      for (int s : pl.tasks[t].succs)
        if (--indeg[s] == 0) ready.push_back(s);
    }
    if (done != n) return fail(HICCL_ERR_STATE, "dependency graph has a cycle");
    if (o == 0) {
      for (auto& m : merged) {
        const uint8_t* p = reinterpret_cast<const uint8_t*>(m.first);
        first.emplace_back(p, p + (m.second - m.first));
      }
    } else {
      for (size_t i = 0; i < merged.size(); ++i)
        if (std::memcmp(reinterpret_cast<const uint8_t*>(merged[i].first), first[i].data(), first[i].size()))
          return fail(HICCL_ERR_RACE, "results depend on the execution order: a dependency edge is missing");
    }
  }
  return HICCL_SUCCESS;
}

}  // namespace hiccl

// =================================================================== C ABI
using namespace hiccl;

#define CHECK_COMM(comm) \
  if (!(comm)) return fail(HICCL_ERR_INVALID_ARG, "NULL communicator")

extern "C" {

const char* hiccl_last_error(void) { return g_err.c_str(); }

int hiccl_version(void) { return 10000; }

// Default tile (measured best): 32 KiB for stage launches; 64 KiB for the persistent executor, whose
// workgroups stream one tile with four worker waves, and 112 KiB for its fp8 tables, whose workgroups
// have seven worker waves (two passes of 32 scale blocks per wave).
static size_t default_tile_bytes(int mode, int dtype) {
  if (mode == HICCL_EXEC_STAGED) return 32 * 1024;
  return dtype == HICCL_FP8_E4M3 ? 112 * 1024 : 64 * 1024;
}

int hiccl_comm_create(int nranks, int dtype, hiccl_comm_t* out) {
  if (!out) return fail(HICCL_ERR_INVALID_ARG, "NULL output pointer");
  if (nranks < 1) return fail(HICCL_ERR_INVALID_ARG, "nranks must be >= 1");
  if (dtype < HICCL_INT32 || dtype > HICCL_FP8_E4M3) return fail(HICCL_ERR_INVALID_ARG, "unknown dtype");
  auto* h = new (std::nothrow) hiccl_comm_s;
  if (!h) return fail(HICCL_ERR_OOM, "out of host memory");
  h->c.P = nranks;
  h->c.dtype = dtype;
  h->c.hier = {nranks};
  h->c.exec.tile_bytes = default_tile_bytes(h->c.exec.mode, dtype);
  *out = h;
  return HICCL_SUCCESS;
}

int hiccl_comm_destroy(hiccl_comm_t comm) {
  delete comm;
  return HICCL_SUCCESS;
}

static int prim_ranges(const Comm& c, const Prim& p, std::vector<Range>& out) {
  out.clear();
  size_t es = elem_size(c.dtype);
  uint64_t nb = p.count * es;
  bool fp8 = c.dtype == HICCL_FP8_E4M3;
  uint64_t nsb = fp8 ? (p.count / kFp8Block) * sizeof(float) : 0;
  auto add = [&](const hiccl_buf_t& b, bool w) {
    uint64_t a = uint64_t(reinterpret_cast<uintptr_t>(b.data));
    out.push_back({0, a, a + nb, w});
    if (fp8) {
      uint64_t s = uint64_t(reinterpret_cast<uintptr_t>(b.scales));
      out.push_back({0, s, s + nsb, w});
    }
  };
  if (p.kind == 0) {
    add(p.send[p.root], false);
    for (int j : p.leaves)
      if (!(j == p.root && p.send[j].data == p.recv[j].data)) add(p.recv[j], true);
  } else {
    for (int i : p.leaves) add(p.send[i], false);
    add(p.recv[p.root], true);
  }
  return 0;
}

static bool overlap(const Range& a, const Range& b) {
  return a.lo < b.hi && b.lo < a.hi && a.hi > a.lo && b.hi > b.lo;
}

static int add_prim(hiccl_comm_t comm, int kind, const hiccl_buf_t* send, const hiccl_buf_t* recv, size_t count,
                    int root, const int* leaves, int nleaves, int op) {
  CHECK_COMM(comm);
  Comm& c = comm->c;
  if (c.planned) return fail(HICCL_ERR_STATE, "cannot register primitives after hiccl_init");
  if (!send || !recv) return fail(HICCL_ERR_INVALID_ARG, "send and recv arrays are required");
  if (root < 0 || root >= c.P) return fail(HICCL_ERR_INVALID_ARG, "root rank out of range");
  if (nleaves < 0 || (nleaves > 0 && !leaves)) return fail(HICCL_ERR_INVALID_ARG, "bad leaf vector");
  if (op < HICCL_SUM || op > HICCL_MIN) return fail(HICCL_ERR_INVALID_ARG, "unknown reduction operator");
  if (kind == 1 && op != HICCL_SUM && (c.dtype == HICCL_BFLOAT16 || c.dtype == HICCL_FP8_E4M3))
    return fail(HICCL_ERR_UNSUPPORTED, "bf16 and fp8 payloads support the sum only");
  if (c.dtype == HICCL_FP8_E4M3 && count % kFp8Block)
    return fail(HICCL_ERR_INVALID_ARG, "fp8 count must be a multiple of 256 (whole scale blocks)");
  Prim p;
  p.kind = kind;
  p.root = root;
  p.count = count;
  p.op = op;
  p.step = c.step;
  std::set<int> seen;
  for (int i = 0; i < nleaves; ++i) {
    int x = leaves[i];
    if (x < 0 || x >= c.P) return fail(HICCL_ERR_INVALID_ARG, "leaf rank out of range");
    if (!seen.insert(x).second) return fail(HICCL_ERR_INVALID_ARG, "duplicate leaf rank");
    p.leaves.push_back(x);
  }
  p.send.assign(send, send + c.P);
  p.recv.assign(recv, recv + c.P);
  if (count > 0) {
    auto need = [&](const hiccl_buf_t& b, const char* what) -> int {
      if (!b.data) return fail(HICCL_ERR_INVALID_ARG, std::string("NULL ") + what + " buffer");
      if (c.dtype == HICCL_FP8_E4M3 && !b.scales)
        return fail(HICCL_ERR_INVALID_ARG, std::string("fp8 ") + what + " buffer needs scales");
      return 0;
    };
    if (kind == 0) {
      if (int rc = need(p.send[root], "send")) return rc;
      for (int j : p.leaves)
        if (int rc = need(p.recv[j], "recv")) return rc;
    } else {
      for (int i : p.leaves)
        if (int rc = need(p.send[i], "send")) return rc;
      if (int rc = need(p.recv[root], "recv")) return rc;
    }
  }
  std::vector<Range> mine, other;
  prim_ranges(c, p, mine);
  // inside one primitive: written ranges must be disjoint from each other,
  // and from read ranges except an exact in-place alias
  for (size_t a = 0; a < mine.size(); ++a)
    for (size_t b = a + 1; b < mine.size(); ++b)
      if ((mine[a].write || mine[b].write) && overlap(mine[a], mine[b])) {
        bool exact = mine[a].lo == mine[b].lo && mine[a].hi == mine[b].hi;
        bool inplace_ok = exact && (mine[a].write != mine[b].write);
        if (!inplace_ok) return fail(HICCL_ERR_INVALID_ARG, "buffers of one primitive overlap");
      }
  // against the other primitives of the current step (Sec. 3.2: concurrent
  // primitives racing on memory have no defined result; rejected here)
  for (const Prim& q : c.prims) {
    if (q.step != c.step) continue;
    prim_ranges(c, q, other);
    for (const Range& a : mine)
      for (const Range& b : other)
        if ((a.write || b.write) && overlap(a, b))
          return fail(HICCL_ERR_RACE, "primitive overlaps another primitive of the same step (add a fence)");
  }
  c.prims.push_back(std::move(p));
  return HICCL_SUCCESS;
}

}  // extern "C"

namespace hiccl {

// Caller memory a communicator touches: the union of its primitives' ranges
// (data and fp8 scales), plus the workspace the plan needs. This is what a
// request keeps resident while it is served.
uint64_t comm_footprint(const Comm& c) {
  std::vector<Range> all, one;
  for (const Prim& p : c.prims) {
    if (p.count == 0 || p.leaves.empty()) continue;
    prim_ranges(c, p, one);
    all.insert(all.end(), one.begin(), one.end());
  }
  std::sort(all.begin(), all.end(), [](const Range& a, const Range& b) { return a.lo < b.lo; });
  uint64_t total = 0, lo = 0, hi = 0;
  bool open = false;
  for (const Range& r : all) {
    if (r.hi <= r.lo) continue;
    if (open && r.lo <= hi) {
      hi = std::max(hi, r.hi);
      continue;
    }
    if (open) total += hi - lo;
    lo = r.lo;
    hi = r.hi;
    open = true;
  }
  if (open) total += hi - lo;
  return total + (c.planned ? c.plan.ws_bytes : 0);
}

// Members of one batch run at the same time with no ordering between them,
// so their memory must not conflict: no communicator twice (one workspace,
// one set of counters), and no member may write caller memory that another
// member reads or writes. Read-read sharing is allowed. A caller-provided
// workspace counts as memory its member writes. One sweep over all ranges
// sorted by start, keeping for reads and for writes the furthest end reached
// by the two members that reach furthest.
int batch_members_disjoint(const std::vector<const Comm*>& comms) {
  for (size_t a = 0; a < comms.size(); ++a)
    for (size_t b = a + 1; b < comms.size(); ++b)
      if (comms[a] == comms[b]) return fail(HICCL_ERR_INVALID_ARG, "a communicator appears twice in one batch");
  struct Tagged {
    Range r;
    int member;
  };
  std::vector<Tagged> all;
  std::vector<Range> one;
  for (size_t m = 0; m < comms.size(); ++m) {
    const Comm& c = *comms[m];
    for (const Prim& p : c.prims) {
      if (p.count == 0 || p.leaves.empty()) continue;
      prim_ranges(c, p, one);
      for (const Range& r : one) all.push_back({r, int(m)});
    }
    if (c.user_ws && c.planned && c.plan.ws_bytes) {
      const uint64_t w = uint64_t(reinterpret_cast<uintptr_t>(c.user_ws));
      all.push_back({Range{0, w, w + c.plan.ws_bytes, true}, int(m)});
    }
  }
  std::sort(all.begin(), all.end(), [](const Tagged& a, const Tagged& b) { return a.r.lo < b.r.lo; });
  struct Reach {
    uint64_t hi[2] = {0, 0};
    int member[2] = {-1, -1};
    void add(uint64_t h, int m) {
      if (m == member[0]) {
        hi[0] = std::max(hi[0], h);
      } else if (m == member[1]) {
        hi[1] = std::max(hi[1], h);
        if (hi[1] > hi[0]) {
          std::swap(hi[0], hi[1]);
          std::swap(member[0], member[1]);
        }
      } else if (h > hi[0]) {
        hi[1] = hi[0];
        member[1] = member[0];
        hi[0] = h;
        member[0] = m;
      } else if (h > hi[1]) {
        hi[1] = h;
        member[1] = m;
      }
    }
    uint64_t other_than(int m) const { return member[0] != m ? hi[0] : hi[1]; }
  } reads, writes;
  for (const Tagged& t : all) {
    if (t.r.hi <= t.r.lo) continue;
    const bool hit = writes.other_than(t.member) > t.r.lo || (t.r.write && reads.other_than(t.member) > t.r.lo);
    if (hit)
      return fail(HICCL_ERR_INVALID_ARG,
                  "batch members conflict: one writes memory that another reads or writes (they run unordered)");
    (t.r.write ? writes : reads).add(t.r.hi, t.member);
  }
  return HICCL_SUCCESS;
}

}  // namespace hiccl

extern "C" {

int hiccl_add_multicast(hiccl_comm_t comm, const hiccl_buf_t* send, const hiccl_buf_t* recv, size_t count, int root,
                        const int* leaves, int nleaves) {
  return add_prim(comm, 0, send, recv, count, root, leaves, nleaves, HICCL_SUM);
}

int hiccl_add_reduction(hiccl_comm_t comm, const hiccl_buf_t* send, const hiccl_buf_t* recv, size_t count,
                        const int* leaves, int nleaves, int root, int op) {
  return add_prim(comm, 1, send, recv, count, root, leaves, nleaves, op);
}

int hiccl_add_fence(hiccl_comm_t comm) {
  CHECK_COMM(comm);
  if (comm->c.planned) return fail(HICCL_ERR_STATE, "cannot add a fence after hiccl_init");
  comm->c.step += 1;
  return HICCL_SUCCESS;
}

static void drop_static(Comm& c) {
  if (c.stat) {
    static_state_free(c.stat);
    c.stat = nullptr;
  }
  c.last_static = false;
}

static void unplan(Comm& c) {
  c.planned = false;
  c.plan = Plan();
  if (c.dev) {
    device_state_free(c.dev);
    c.dev = nullptr;
  }
  drop_static(c);
}

int hiccl_set_hierarchy(hiccl_comm_t comm, const int* factors, int nlevels) {
  CHECK_COMM(comm);
  if (!factors || nlevels < 1) return fail(HICCL_ERR_INVALID_ARG, "hierarchy needs at least one factor");
  long prod = 1;
  for (int i = 0; i < nlevels; ++i) {
    if (factors[i] < 1) return fail(HICCL_ERR_INVALID_ARG, "hierarchy factors must be >= 1");
    prod *= factors[i];
  }
  if (prod != comm->c.P) return fail(HICCL_ERR_INVALID_ARG, "product of hierarchy factors must equal nranks");
  unplan(comm->c);
  comm->c.hier.assign(factors, factors + nlevels);
  return HICCL_SUCCESS;
}

int hiccl_set_stripe(hiccl_comm_t comm, int s) {
  CHECK_COMM(comm);
  if (s < 1) return fail(HICCL_ERR_INVALID_ARG, "stripe must be >= 1");
  unplan(comm->c);
  comm->c.stripe = s;
  return HICCL_SUCCESS;
}

int hiccl_set_ring(hiccl_comm_t comm, int n) {
  CHECK_COMM(comm);
  if (n < 1) return fail(HICCL_ERR_INVALID_ARG, "ring must be >= 1");
  unplan(comm->c);
  comm->c.ring = n;
  return HICCL_SUCCESS;
}

int hiccl_set_pipeline(hiccl_comm_t comm, int m) {
  CHECK_COMM(comm);
  if (m < 1) return fail(HICCL_ERR_INVALID_ARG, "pipeline must be >= 1");
  unplan(comm->c);
  comm->c.pipe = m;
  return HICCL_SUCCESS;
}

int hiccl_set_share(hiccl_comm_t comm, int rank) {
  CHECK_COMM(comm);
  if (rank < -1 || rank >= comm->c.P) return fail(HICCL_ERR_INVALID_ARG, "share rank must be -1 or a rank");
  unplan(comm->c);
  comm->c.share = rank;
  return HICCL_SUCCESS;
}

int hiccl_set_exec(hiccl_comm_t comm, int mode, size_t tile_bytes, int grid, int order) {
  CHECK_COMM(comm);
  if (mode != HICCL_EXEC_PERSISTENT && mode != HICCL_EXEC_STAGED) return fail(HICCL_ERR_INVALID_ARG, "bad mode");
  if (order < HICCL_ORDER_STAGE || order > HICCL_ORDER_CRITICAL) return fail(HICCL_ERR_INVALID_ARG, "bad order");
  if (grid < 0) return fail(HICCL_ERR_INVALID_ARG, "grid must be >= 0");
  if (tile_bytes != 0 && (tile_bytes < 256 || tile_bytes > (size_t(1) << 30)))
    return fail(HICCL_ERR_INVALID_ARG, "tile must be 256 bytes .. 1 GiB");   // device offsets are 32-bit
  unplan(comm->c);
  comm->c.exec.mode = mode;
  // default tile: 64 KiB for the persistent executor, 32 KiB for stage launches (measured best)
  comm->c.exec.tile_bytes = tile_bytes ? tile_bytes : default_tile_bytes(mode, comm->c.dtype);
  comm->c.exec.grid = grid;
  comm->c.exec.order = order;
  return HICCL_SUCCESS;
}

int hiccl_set_claim(hiccl_comm_t comm, int queues, int batch) {
  CHECK_COMM(comm);
  if (queues < 0 || queues > 8 || batch < 0 || batch > 1024)
    return fail(HICCL_ERR_INVALID_ARG, "queues must be 0..8 and batch 0..1024");
  comm->c.exec.queues = queues ? queues : 8;
  comm->c.exec.batch = batch ? batch : 4;
  if (comm->c.dev) {
    device_state_free(comm->c.dev);
    comm->c.dev = nullptr;
  }
  drop_static(comm->c);
  return HICCL_SUCCESS;
}

int hiccl_set_trace(hiccl_comm_t comm, int on) {
  CHECK_COMM(comm);
  if (on != 0 && on != 1) return fail(HICCL_ERR_INVALID_ARG, "trace must be 0 or 1");
  if (comm->c.exec.trace == (on != 0)) return HICCL_SUCCESS;
  comm->c.exec.trace = on != 0;
  if (comm->c.dev) {             // the next run uploads the tables with (or without) the trace buffer
    device_state_free(comm->c.dev);
    comm->c.dev = nullptr;
  }
  drop_static(comm->c);
  return HICCL_SUCCESS;
}

int hiccl_set_spin_limit(hiccl_comm_t comm, uint32_t polls) {
  CHECK_COMM(comm);
  if (polls == 0) return fail(HICCL_ERR_INVALID_ARG, "spin limit must be >= 1");
  comm->c.exec.spin_limit = polls;
  device_state_set_spin_limit(comm->c.dev, polls);   // uploaded tables and counters stay
  return HICCL_SUCCESS;
}

int hiccl_init(hiccl_comm_t comm) {
  CHECK_COMM(comm);
  Comm& c = comm->c;
  if (c.planned) return fail(HICCL_ERR_STATE, "communicator already initialized");
  int rc = build_plan(c);
  if (rc) return rc;
  c.planned = true;
  return HICCL_SUCCESS;
}

int hiccl_workspace_size(hiccl_comm_t comm, size_t* bytes) {
  CHECK_COMM(comm);
  if (!comm->c.planned) return fail(HICCL_ERR_STATE, "call hiccl_init first");
  if (!bytes) return fail(HICCL_ERR_INVALID_ARG, "NULL output");
  *bytes = comm->c.plan.ws_bytes;
  return HICCL_SUCCESS;
}

int hiccl_set_workspace(hiccl_comm_t comm, void* dptr, size_t bytes) {
  CHECK_COMM(comm);
  Comm& c = comm->c;
  if (!c.planned) return fail(HICCL_ERR_STATE, "call hiccl_init first");
  if (bytes < c.plan.ws_bytes) return fail(HICCL_ERR_INVALID_ARG, "workspace smaller than hiccl_workspace_size");
  if (reinterpret_cast<uintptr_t>(dptr) % 256) return fail(HICCL_ERR_INVALID_ARG, "workspace must be 256-byte aligned");
  if (c.dev) {
    device_state_free(c.dev);
    c.dev = nullptr;
  }
  c.user_ws = dptr;
  c.user_ws_bytes = bytes;
  return HICCL_SUCCESS;
}

int hiccl_query_bytes(hiccl_comm_t comm, const int* acct, int nacct, uint64_t* level_bytes, uint64_t* hbm_read,
                      uint64_t* hbm_written) {
  CHECK_COMM(comm);
  const Comm& c = comm->c;
  if (!c.planned) return fail(HICCL_ERR_STATE, "call hiccl_init first");
  std::vector<int> h = c.hier;
  if (acct && nacct > 0) {
    long prod = 1;
    for (int i = 0; i < nacct; ++i) {
      if (acct[i] < 1) return fail(HICCL_ERR_INVALID_ARG, "accounting factors must be >= 1");
      prod *= acct[i];
    }
    if (prod != c.P) return fail(HICCL_ERR_INVALID_ARG, "accounting hierarchy must multiply to nranks");
    h.assign(acct, acct + nacct);
  }
  if (level_bytes) {
    std::vector<uint64_t> lb(h.size() + 1, 0);
    for (const Task& t : c.plan.tasks) {
      uint64_t nb = t.count * elem_size(t.dtype);
      if (t.dtype == HICCL_FP8_E4M3) nb += (t.count / kFp8Block) * sizeof(float);
      if (t.kind == kCopy) {
        lb[hier_depth(t.src_rank[0], t.dst_rank, h)] += nb;
      } else {
        for (int r : t.src_rank)
          if (r != t.dst_rank) lb[hier_depth(r, t.dst_rank, h)] += nb;
      }
    }
    std::copy(lb.begin(), lb.end(), level_bytes);
  }
  if (hbm_read) *hbm_read = c.plan.hbm_read;
  if (hbm_written) *hbm_written = c.plan.hbm_written;
  return HICCL_SUCCESS;
}

int hiccl_plan_info(hiccl_comm_t comm, hiccl_plan_info_t* info) {
  CHECK_COMM(comm);
  const Comm& c = comm->c;
  if (!c.planned) return fail(HICCL_ERR_STATE, "call hiccl_init first");
  if (!info) return fail(HICCL_ERR_INVALID_ARG, "NULL output");
  info->ntasks = c.plan.tasks.size();
  info->ntiles = c.plan.tile_task.size();
  info->nedges = c.plan.nedges;
  info->nstages = uint64_t(c.plan.nstages);
  info->workspace_bytes = c.plan.ws_bytes;
  info->hbm_read = c.plan.hbm_read;
  info->hbm_written = c.plan.hbm_written;
  info->tile_elems = tile_elems_for(c.exec.tile_bytes, c.dtype);
  return HICCL_SUCCESS;
}

int hiccl_plan_tasks(hiccl_comm_t comm, hiccl_task_info_t* out, size_t cap, size_t* n) {
  CHECK_COMM(comm);
  const Comm& c = comm->c;
  if (!c.planned) return fail(HICCL_ERR_STATE, "call hiccl_init first");
  size_t m = std::min(cap, c.plan.tasks.size());
  if (m && !out) return fail(HICCL_ERR_INVALID_ARG, "NULL output");
  for (size_t i = 0; i < m; ++i) {
    const Task& t = c.plan.tasks[i];
    hiccl_task_info_t& o = out[i];
    std::memset(&o, 0, sizeof(o));
    o.kind = t.kind;
    o.prim = t.prim;
    o.step = t.step;
    o.stripe = t.stripe;
    o.channel = t.channel;
    o.stage = t.stage;
    o.dst_rank = t.dst_rank;
    o.dst_workspace = t.dst_ws ? 1 : 0;
    o.nsrc = int(t.src_rank.size());
    for (int k = 0; k < o.nsrc && k < HICCL_INFO_MAX_SRC; ++k) o.src_rank[k] = t.src_rank[k];
    o.npred = int(t.preds.size());
    o.ring_step = t.ring_step;
    o.count = t.count;
    o.offset = t.offset;
  }
  if (n) *n = c.plan.tasks.size();
  return HICCL_SUCCESS;
}

int hiccl_plan_edges(hiccl_comm_t comm, uint32_t* from, uint32_t* to, size_t cap, size_t* n) {
  CHECK_COMM(comm);
  const Comm& c = comm->c;
  if (!c.planned) return fail(HICCL_ERR_STATE, "call hiccl_init first");
  size_t total = 0;
  for (const Task& t : c.plan.tasks) total += t.preds.size();
  if (std::min(cap, total) && (!from || !to)) return fail(HICCL_ERR_INVALID_ARG, "NULL output");
  size_t m = 0;
  for (size_t i = 0; i < c.plan.tasks.size() && m < cap; ++i)
    for (int p : c.plan.tasks[i].preds) {
      if (m == cap) break;
      from[m] = uint32_t(p);
      to[m] = uint32_t(i);
      ++m;
    }
  if (n) *n = total;
  return HICCL_SUCCESS;
}

int hiccl_validate_host(hiccl_comm_t comm, uint64_t seed, int norders) {
  CHECK_COMM(comm);
  if (!comm->c.planned) return fail(HICCL_ERR_STATE, "call hiccl_init first");
  if (comm->c.share >= 0) return fail(HICCL_ERR_STATE, "the schedule check needs the whole plan, not one rank's share");
  return validate_host(comm->c, seed, norders);
}

}  // extern "C"
