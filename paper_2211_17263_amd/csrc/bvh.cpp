// Host BVH builder: surface-area heuristic (16 bins per axis, an exact sweep
// over sorted centroids for small ranges), leaves of at most 4 triangles, a
// range of at most 4 kept as a leaf only when no split is cheaper under the
// SAH, and inner-node depth bounded by kMaxInnerDepth: a split is admissible
// only if both children still fit a balanced subtree in the depth that remains
// (else object median).  The binary tree is then collapsed into the 4-wide
// device layout (each node takes its grandchildren, or a child that is a leaf,
// as its up to four children), so the device depth is at most kMaxDepth4 and
// the traversal stack bound holds.  Output is appended to flat node/triangle
// arrays in the 128-byte / 48-byte layouts the kernels read with 16-byte loads.
#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstring>
#include <limits>
#include <vector>

#include "prdpt_internal.h"

namespace prdpt {

namespace {

struct Box {
  float lo[3] = {FLT_MAX, FLT_MAX, FLT_MAX};
  float hi[3] = {-FLT_MAX, -FLT_MAX, -FLT_MAX};
  void grow(const Box& b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], b.lo[a]);
      hi[a] = std::max(hi[a], b.hi[a]);
    }
  }
  void grow(const float* p) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
  double area() const {
    if (lo[0] > hi[0]) return 0.0;
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

// binary node of the build (host only): both children's padded boxes, child
// index and leaf count (cnt > 0: idx is the first of cnt triangles)
struct Node2 {
  float lo[2][3], hi[2][3];
  int32_t idx[2], cnt[2];
};

struct Prim {
  Box box;
  float c[3];
  int32_t tri;  // index into the caller's triangle array
};

constexpr int kBins = 16;
constexpr int kSweepMax = 32;   // ranges up to this size use the exact sweep

// SAH costs: one node visit (both child boxes) and one triangle test
#ifndef PRDPT_SAH_NODE
#define PRDPT_SAH_NODE 2.0
#endif
#ifndef PRDPT_SAH_TRI
#define PRDPT_SAH_TRI 1.0
#endif
constexpr double kCostNode = PRDPT_SAH_NODE;
constexpr double kCostTri = PRDPT_SAH_TRI;

// largest triangle count a subtree whose root inner node sits at depth D can
// hold within the depth bound (two leaves of kLeafMax at depth kMaxInnerDepth);
// below the bound (the children of a leaf) nothing fits
inline long long capacity(int D) {
  const int levels = kMaxInnerDepth - D + 1;
  if (levels < 0) return 0;
  return levels >= 40 ? (1LL << 50) : (long long)kLeafMax << levels;
}

struct Builder {
  const float* tri9;
  const int32_t* tri_mat;
  int32_t id_base;
  std::vector<Node2>* nodes;
  std::vector<Tri>* tris;
  std::vector<Prim> prims;
  int max_depth = 0;

  // padded copy of a box, rounded outward in binary32
  static void padded(const Box& b, float lo[3], float hi[3]) {
    double mag = 1.0;
    for (int a = 0; a < 3; ++a) mag = std::max({mag, (double)std::fabs(b.lo[a]), (double)std::fabs(b.hi[a])});
    double pad = 1e-4 * mag;
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::nextafter((float)((double)b.lo[a] - pad), -FLT_MAX);
      hi[a] = std::nextafter((float)((double)b.hi[a] + pad), FLT_MAX);
    }
  }

  int emit_leaf(int begin, int end) {
    int first = (int)tris->size();
    for (int i = begin; i < end; ++i) {
      int t = prims[i].tri;
      const float* v = tri9 + 9 * (size_t)t;
      Tri o;
      o.v0x = v[0]; o.v0y = v[1]; o.v0z = v[2];
      o.e1x = v[3] - v[0]; o.e1y = v[4] - v[1]; o.e1z = v[5] - v[2];
      o.e2x = v[6] - v[0]; o.e2y = v[7] - v[1]; o.e2z = v[8] - v[2];
      o.id = id_base + t;
      o.mat = tri_mat[t];
      o.inst = 0;  // set by the caller, which knows the instance
      tris->push_back(o);
    }
    return first;
  }

  Box range_box(int begin, int end) const {
    Box b;
    for (int i = begin; i < end; ++i) b.grow(prims[i].box);
    return b;
  }

  // exact SAH sweep over the centroids sorted along each axis; returns the
  // best cost (sum of child area x count) and sets axis/position, or DBL_MAX
  double sweep(int begin, int end, long long child_cap, int* best_axis, int* best_mid) {
    const int n = end - begin;
    double best = DBL_MAX;
    std::vector<double> right(n);
    for (int a = 0; a < 3; ++a) {
      std::sort(prims.begin() + begin, prims.begin() + end, [&](const Prim& p, const Prim& q) {
        return p.c[a] < q.c[a] || (p.c[a] == q.c[a] && p.tri < q.tri);
      });
      Box acc;
      for (int i = n - 1; i > 0; --i) {
        acc.grow(prims[begin + i].box);
        right[i] = acc.area();
      }
      Box lacc;
      for (int i = 1; i < n; ++i) {
        lacc.grow(prims[begin + i - 1].box);
        if (i > child_cap || n - i > child_cap) continue;
        const double cost = lacc.area() * i + right[i] * (n - i);
        if (cost < best) {
          best = cost;
          *best_axis = a;
          *best_mid = i;
        }
      }
    }
    if (best < DBL_MAX) {
      const int a = *best_axis;
      std::sort(prims.begin() + begin, prims.begin() + end, [&](const Prim& p, const Prim& q) {
        return p.c[a] < q.c[a] || (p.c[a] == q.c[a] && p.tri < q.tri);
      });
    }
    return best;
  }

  // returns (idx, cnt) reference to a subtree: cnt > 0 leaf, cnt == 0 inner
  // node at inner-node depth `depth`
  void build(int begin, int end, int depth, int32_t* idx, int32_t* cnt) {
    int n = end - begin;
    const long long child_cap = capacity(depth + 1);
    if (n == 1) {
      *idx = emit_leaf(begin, end);
      *cnt = n;
      return;
    }
    Box cb;
    for (int i = begin; i < end; ++i) cb.grow(prims[i].c);
    int axis = 0;
    for (int a = 1; a < 3; ++a)
      if (cb.hi[a] - cb.lo[a] > cb.hi[axis] - cb.lo[axis]) axis = a;
    int mid = -1;
    double best = DBL_MAX;
    if (n <= kSweepMax) {
      int ba = -1, bm = -1;
      best = sweep(begin, end, child_cap, &ba, &bm);
      if (best < DBL_MAX) mid = begin + bm;
    } else if (cb.hi[axis] > cb.lo[axis]) {
      int best_axis = -1, best_bin = -1;
      for (int a = 0; a < 3; ++a) {
        float ext = cb.hi[a] - cb.lo[a];
        if (!(ext > 0.0f)) continue;
        Box bb[kBins];
        int bc[kBins] = {0};
        float k = kBins / ext;
        for (int i = begin; i < end; ++i) {
          int b = std::min(kBins - 1, (int)((prims[i].c[a] - cb.lo[a]) * k));
          bb[b].grow(prims[i].box);
          bc[b]++;
        }
        double right_area[kBins];
        int right_cnt[kBins];
        Box acc;
        int cacc = 0;
        for (int b = kBins - 1; b > 0; --b) {
          acc.grow(bb[b]);
          cacc += bc[b];
          right_area[b] = acc.area();
          right_cnt[b] = cacc;
        }
        Box lacc;
        int lcnt = 0;
        for (int b = 0; b < kBins - 1; ++b) {
          lacc.grow(bb[b]);
          lcnt += bc[b];
          if (lcnt == 0 || right_cnt[b + 1] == 0) continue;
          if (lcnt > child_cap || right_cnt[b + 1] > child_cap) continue;
          double cost = lacc.area() * lcnt + right_area[b + 1] * right_cnt[b + 1];
          if (cost < best) {
            best = cost;
            best_axis = a;
            best_bin = b;
          }
        }
      }
      if (best_axis >= 0) {
        int a = best_axis;
        float k = kBins / (cb.hi[a] - cb.lo[a]);
        float lo = cb.lo[a];
        auto it = std::partition(prims.begin() + begin, prims.begin() + end, [&](const Prim& p) {
          return std::min(kBins - 1, (int)((p.c[a] - lo) * k)) <= best_bin;
        });
        mid = (int)(it - prims.begin());
        if (mid == begin || mid == end) mid = -1;
      }
    }
    if (n <= kLeafMax) {
      // keep a leaf unless splitting is cheaper: node visit + expected tests
      const double parent = range_box(begin, end).area();
      // (an inner node here must still respect the depth bound)
      const double split = mid < 0 || !(parent > 0.0) || depth > kMaxInnerDepth
                               ? DBL_MAX
                               : kCostNode + kCostTri * best / parent;
      if (kCostTri * n <= split) {
        *idx = emit_leaf(begin, end);
        *cnt = n;
        return;
      }
    }
    max_depth = std::max(max_depth, depth);
    if (mid < 0) {
      mid = begin + n / 2;
      std::nth_element(prims.begin() + begin, prims.begin() + mid, prims.begin() + end,
                       [&](const Prim& p, const Prim& q) {
                         return p.c[axis] < q.c[axis] || (p.c[axis] == q.c[axis] && p.tri < q.tri);
                       });
    }
    int ni = (int)nodes->size();
    nodes->push_back(Node2{});
    Box lb = range_box(begin, mid), rb = range_box(mid, end);
    int32_t i0, c0, i1, c1;
    build(begin, mid, depth + 1, &i0, &c0);
    build(mid, end, depth + 1, &i1, &c1);
    float llo[3], lhi[3], rlo[3], rhi[3];
    padded(lb, llo, lhi);
    padded(rb, rlo, rhi);
    Node2& nd = (*nodes)[ni];
    for (int a = 0; a < 3; ++a) {
      nd.lo[0][a] = llo[a];
      nd.hi[0][a] = lhi[a];
      nd.lo[1][a] = rlo[a];
      nd.hi[1][a] = rhi[a];
    }
    nd.idx[0] = i0; nd.cnt[0] = c0; nd.idx[1] = i1; nd.cnt[1] = c1;
    *idx = ni;
    *cnt = 0;
  }
};

// Appends the 4-wide node for binary inner node i (and, depth first, its
// subtree) to out; returns its index.
int32_t collapse(const std::vector<Node2>& n2, int i, std::vector<Node>& out) {
  struct Child {
    const float* lo;
    const float* hi;
    int32_t idx, cnt;  // cnt > 0: leaf; cnt == 0: binary inner node idx
  };
  Child ch[4];
  int nc = 0;
  const Node2& b = n2[i];
  for (int s = 0; s < 2; ++s) {
    if (b.idx[s] < 0) continue;  // the missing second child of a wrapped leaf
    if (b.cnt[s] > 0) {
      ch[nc++] = Child{b.lo[s], b.hi[s], b.idx[s], b.cnt[s]};
    } else {
      const Node2& g = n2[b.idx[s]];
      for (int t = 0; t < 2; ++t)
        if (g.idx[t] >= 0) ch[nc++] = Child{g.lo[t], g.hi[t], g.idx[t], g.cnt[t]};
    }
  }
  const int32_t me = (int32_t)out.size();
  out.push_back(Node{});
  int32_t ref[4];
  for (int c = 0; c < 4; ++c) {
    if (c >= nc) {
      ref[c] = kEmptyChild;
    } else if (ch[c].cnt > 0) {
      ref[c] = ~((ch[c].idx << 3) | (ch[c].cnt - 1));
    } else {
      ref[c] = collapse(n2, ch[c].idx, out);
    }
  }
  Node& nd = out[me];
  // an empty slot gets the inverted box lo = +inf, hi = -inf: every slab
  // test misses it, whatever the ray
  const float inf = std::numeric_limits<float>::infinity();
  for (int c = 0; c < 4; ++c) {
    const bool use = c < nc;
    nd.lox[c] = use ? ch[c].lo[0] : inf;
    nd.loy[c] = use ? ch[c].lo[1] : inf;
    nd.loz[c] = use ? ch[c].lo[2] : inf;
    nd.hix[c] = use ? ch[c].hi[0] : -inf;
    nd.hiy[c] = use ? ch[c].hi[1] : -inf;
    nd.hiz[c] = use ? ch[c].hi[2] : -inf;
    nd.ref[c] = ref[c];
    nd.pad[c] = 0;
  }
  return me;
}

}  // namespace

// Builds one instance BVH over triangles `list[0..n)` (indices into tri9).
// The root is always an inner node; depth is that of the 4-wide tree.
BvhOut build_bvh(const float* tri9, const int32_t* tri_mat, const int32_t* list, int n,
                 int32_t id_base, std::vector<Node>& nodes, std::vector<Tri>& tris) {
  std::vector<Node2> n2;
  Builder b;
  b.tri9 = tri9;
  b.tri_mat = tri_mat;
  b.id_base = id_base;
  b.nodes = &n2;
  b.tris = &tris;
  b.prims.resize(n);
  for (int i = 0; i < n; ++i) {
    Prim& p = b.prims[i];
    const float* v = tri9 + 9 * (size_t)list[i];
    p.box.grow(v);
    p.box.grow(v + 3);
    p.box.grow(v + 6);
    for (int a = 0; a < 3; ++a) p.c[a] = (p.box.lo[a] + p.box.hi[a]) * 0.5f;
    p.tri = list[i];
  }
  BvhOut out{-1, 0};
  if (n == 0) return out;
  int32_t idx, cnt;
  if ((long long)n > capacity(1)) return BvhOut{-2, 0};
  b.build(0, n, 1, &idx, &cnt);
  if (cnt > 0) {  // a single leaf: wrap it in a root with one child
    int ni = (int)n2.size();
    Node2 nd{};
    float lo[3], hi[3];
    Builder::padded(b.range_box(0, n), lo, hi);
    for (int a = 0; a < 3; ++a) {
      nd.lo[0][a] = lo[a];
      nd.hi[0][a] = hi[a];
    }
    nd.idx[0] = idx; nd.cnt[0] = cnt; nd.idx[1] = -1; nd.cnt[1] = 0;
    n2.push_back(nd);
    idx = ni;
    b.max_depth = 1;
  }
  out.root = collapse(n2, idx, nodes);
  out.depth = (b.max_depth + 1) / 2;
  return out;
}

}  // namespace prdpt
