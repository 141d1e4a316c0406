// Host-side construction of the 4-wide BVH (binned SAH binary tree, collapsed to 4 children
// per node) and of the hemi-octahedral cell moment table.
#include "gi_host.hpp"

#include <algorithm>
#include <atomic>
#include <stdexcept>
#include <cmath>
#include <cstring>
#include <future>
#include <numeric>
#include <thread>

namespace gi {

namespace {

struct Box {
  float lo[3] = {3.0e38f, 3.0e38f, 3.0e38f};
  float hi[3] = {-3.0e38f, -3.0e38f, -3.0e38f};
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
    double dx = hi[0] - lo[0], dy = hi[1] - lo[1], dz = hi[2] - lo[2];
    if (dx < 0 || dy < 0 || dz < 0) return 0.0;
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

struct BinNode {
  Box box;
  int32_t left = -1, right = -1;   // children in the binary node array (inner)
  uint32_t count = 0;              // leaf: number of triangles
  uint32_t tri[2] = {0, 0};        // leaf: triangle indices
};

// A reference: one triangle, or the part of it inside a region of space left by spatial
// splits, with a box that contains that part.
struct Ref {
  Box box;
  uint32_t tri;
};

// the float at or below / at or above a double
inline float round_down(double x) {
  const float f = (float)x;
  return (double)f > x ? std::nextafter(f, -INFINITY) : f;
}
inline float round_up(double x) {
  const float f = (float)x;
  return (double)f < x ? std::nextafter(f, INFINITY) : f;
}

inline bool empty(const Box& b) { return b.lo[0] > b.hi[0] || b.lo[1] > b.hi[1] || b.lo[2] > b.hi[2]; }

inline Box intersect(const Box& a, const Box& b) {
  Box r;
  for (int k = 0; k < 3; ++k) {
    r.lo[k] = std::max(a.lo[k], b.lo[k]);
    r.hi[k] = std::min(a.hi[k], b.hi[k]);
  }
  return r;
}

// Binned SAH binary tree with spatial splits (Stich, Friedrich and Dietrich 2009).  Where the
// best object split leaves children whose boxes overlap by more than a small fraction of the
// scene's area, splitting space at a plane is tried as well: triangles that straddle the plane
// go to both sides, each with the box of its part on that side.  Those boxes are computed in
// double and rounded outward, so every point of a triangle lies in the box of one of its
// references, and a conservative walk finds every hit.
struct Builder {
  const float* tv;                 // [n][9]
  std::vector<BinNode> nodes;
  std::mutex mu;
  double min_overlap = 0.0;        // overlap area above which spatial splits are tried

  static constexpr int kBins = 64;
  static constexpr int kSpatialBins = 32;
  static constexpr uint32_t kLeafMax = 2;

  struct Split {
    double cost = 1e300;
    int axis = -1;
    int bin = -1;
    float pos = 0.0f;
    Box lbox, rbox;
  };

  int32_t alloc_pair() {
    std::lock_guard<std::mutex> g(mu);
    nodes.emplace_back();
    nodes.emplace_back();
    return (int32_t)nodes.size() - 2;
  }

  // boxes of the parts of reference r on either side of the plane x_a = pos
  void clip(const Ref& r, int a, float pos, Box& lb, Box& rb) const {
    lb = Box();
    rb = Box();
    const float* v = tv + 9 * (size_t)r.tri;
    for (int e = 0; e < 3; ++e) {
      const float* p = v + 3 * e;
      const float* q = v + 3 * ((e + 1) % 3);
      if (p[a] <= pos) lb.grow(p);
      if (p[a] >= pos) rb.grow(p);
      if ((p[a] < pos && q[a] > pos) || (p[a] > pos && q[a] < pos)) {
        const double t = ((double)pos - p[a]) / ((double)q[a] - p[a]);
        Box x;
        for (int k = 0; k < 3; ++k) {
          if (k == a) {
            x.lo[k] = x.hi[k] = pos;
          } else {
            const double c = p[k] + t * ((double)q[k] - p[k]);
            x.lo[k] = round_down(c);
            x.hi[k] = round_up(c);
          }
        }
        lb.grow(x);
        rb.grow(x);
      }
    }
    lb = intersect(lb, r.box);
    rb = intersect(rb, r.box);
    lb.hi[a] = std::min(lb.hi[a], pos);
    rb.lo[a] = std::max(rb.lo[a], pos);
  }

  // binned SAH over the centroids of the reference boxes, all three axes
  Split object_split(const std::vector<Ref>& refs, const Box& cbox) const {
    Split best;
    for (int a = 0; a < 3; ++a) {
      const float ext = cbox.hi[a] - cbox.lo[a];
      if (!(ext > 0.0f)) continue;
      Box bb[kBins];
      uint32_t bc[kBins] = {0};
      const double k = kBins / (double)ext * (1.0 - 1e-6);
      for (const Ref& r : refs) {
        const float c = (r.box.lo[a] + r.box.hi[a]) * 0.5f;
        int b = (int)((c - cbox.lo[a]) * k);
        b = std::min(std::max(b, 0), kBins - 1);
        bb[b].grow(r.box);
        bc[b]++;
      }
      Box lb[kBins];
      uint32_t lc[kBins];
      Box acc;
      uint32_t c = 0;
      for (int b = 0; b < kBins; ++b) {
        acc.grow(bb[b]);
        c += bc[b];
        lb[b] = acc;
        lc[b] = c;
      }
      Box racc;
      uint32_t rc = 0;
      for (int b = kBins - 1; b >= 1; --b) {
        racc.grow(bb[b]);
        rc += bc[b];
        const uint32_t l = lc[b - 1];
        if (l == 0 || rc == 0) continue;
        const double cost = lb[b - 1].area() * l + racc.area() * rc;
        if (cost < best.cost) {
          best.cost = cost;
          best.axis = a;
          best.bin = b;
          best.lbox = lb[b - 1];
          best.rbox = racc;
        }
      }
    }
    return best;
  }

  // spatial bins over the node's box: each reference is chopped into the bins it spans
  Split spatial_split(const std::vector<Ref>& refs, const Box& box) const {
    Split best;
    for (int a = 0; a < 3; ++a) {
      const float lo = box.lo[a], ext = box.hi[a] - box.lo[a];
      if (!(ext > 0.0f)) continue;
      float pos[kSpatialBins + 1];
      for (int b = 0; b <= kSpatialBins; ++b) pos[b] = lo + ext * ((float)b / (float)kSpatialBins);
      pos[kSpatialBins] = box.hi[a];
      const double k = kSpatialBins / (double)ext;
      auto bin_of = [&](float x) { return std::min(std::max((int)((x - lo) * k), 0), kSpatialBins - 1); };
      Box bb[kSpatialBins];
      uint32_t enter[kSpatialBins] = {0}, leave[kSpatialBins] = {0};
      for (const Ref& r : refs) {
        const int b0 = bin_of(r.box.lo[a]), b1 = bin_of(r.box.hi[a]);
        Ref cur = r;
        for (int b = b0; b < b1; ++b) {
          Box l, rr;
          clip(cur, a, pos[b + 1], l, rr);
          if (!empty(l)) bb[b].grow(l);
          cur.box = rr;
        }
        if (!empty(cur.box)) bb[b1].grow(cur.box);
        enter[b0]++;
        leave[b1]++;
      }
      Box lb[kSpatialBins];
      uint32_t lc[kSpatialBins];
      Box acc;
      uint32_t c = 0;
      for (int b = 0; b < kSpatialBins; ++b) {
        acc.grow(bb[b]);
        c += enter[b];
        lb[b] = acc;
        lc[b] = c;
      }
      Box racc;
      uint32_t rc = 0;
      for (int b = kSpatialBins - 1; b >= 1; --b) {
        racc.grow(bb[b]);
        rc += leave[b];
        const uint32_t l = lc[b - 1];
        if (l == 0 || rc == 0) continue;
        const double cost = lb[b - 1].area() * l + racc.area() * rc;
        if (cost < best.cost) {
          best.cost = cost;
          best.axis = a;
          best.bin = b;
          best.pos = pos[b];
          best.lbox = lb[b - 1];
          best.rbox = racc;
        }
      }
    }
    return best;
  }

  // splits refs by the plane, spending the references it adds from budget; false (refs
  // untouched) if the budget is too small or one side would keep every reference
  bool apply_spatial(std::vector<Ref>& refs, const Split& sp, std::vector<Ref>& left, std::vector<Ref>& right,
                     int64_t& budget) const {
    const int a = sp.axis;
    int64_t extra = 0;
    for (const Ref& r : refs) extra += r.box.lo[a] < sp.pos && r.box.hi[a] > sp.pos;
    if (extra > budget) return false;
    left.clear();
    right.clear();
    for (const Ref& r : refs) {
      if (r.box.hi[a] <= sp.pos) {
        left.push_back(r);
      } else if (r.box.lo[a] >= sp.pos) {
        right.push_back(r);
      } else {
        Box lb, rb;
        clip(r, a, sp.pos, lb, rb);
        if (!empty(lb)) left.push_back(Ref{lb, r.tri});
        if (!empty(rb)) right.push_back(Ref{rb, r.tri});
      }
    }
    if (left.size() == refs.size() || right.size() == refs.size() || left.empty() || right.empty()) return false;
    budget -= (int64_t)(left.size() + right.size() - refs.size());
    return true;
  }

  // builds node ni over refs (consumed); budget: references spatial splits in this subtree may
  // add (handed to the children in proportion to their references, so the tree does not depend
  // on the order in which threads build subtrees)
  void build(int32_t ni, std::vector<Ref>& refs, int depth, int64_t budget) {
    Box box, cbox;
    for (const Ref& r : refs) {
      box.grow(r.box);
      const float c[3] = {(r.box.lo[0] + r.box.hi[0]) * 0.5f, (r.box.lo[1] + r.box.hi[1]) * 0.5f,
                          (r.box.lo[2] + r.box.hi[2]) * 0.5f};
      cbox.grow(c);
    }
    BinNode node;
    node.box = box;
    if (refs.size() <= kLeafMax) {
      node.count = (uint32_t)refs.size();
      for (uint32_t i = 0; i < node.count; ++i) node.tri[i] = refs[i].tri;
      std::lock_guard<std::mutex> g(mu);
      nodes[ni] = node;
      return;
    }
    const Split os = object_split(refs, cbox);
    std::vector<Ref> left, right;
    bool done = false;
    if (os.axis >= 0 && budget > 0 && intersect(os.lbox, os.rbox).area() > min_overlap &&
        !empty(intersect(os.lbox, os.rbox))) {
      const Split ss = spatial_split(refs, box);
      if (ss.axis >= 0 && ss.cost < os.cost) done = apply_spatial(refs, ss, left, right, budget);
    }
    if (!done) {
      left.clear();
      right.clear();
      if (os.axis < 0) {
        // all centroids coincide: split the list in half
        const size_t h = refs.size() / 2;
        left.assign(refs.begin(), refs.begin() + h);
        right.assign(refs.begin() + h, refs.end());
      } else {
        const int a = os.axis;
        const float ext = cbox.hi[a] - cbox.lo[a];
        const double k = kBins / (double)ext * (1.0 - 1e-6);
        for (const Ref& r : refs) {
          const float c = (r.box.lo[a] + r.box.hi[a]) * 0.5f;
          int b = (int)((c - cbox.lo[a]) * k);
          b = std::min(std::max(b, 0), kBins - 1);
          (b < os.bin ? left : right).push_back(r);
        }
        if (left.empty() || right.empty()) {
          left.clear();
          right.clear();
          const size_t h = refs.size() / 2;
          left.assign(refs.begin(), refs.begin() + h);
          right.assign(refs.begin() + h, refs.end());
        }
      }
    }
    std::vector<Ref>().swap(refs);
    const int32_t l = alloc_pair();
    node.left = l;
    node.right = l + 1;
    {
      std::lock_guard<std::mutex> g(mu);
      nodes[ni] = node;
    }
    const int64_t bl = budget * (int64_t)left.size() / (int64_t)(left.size() + right.size());
    const int64_t br = budget - bl;
    if (left.size() + right.size() > 200000 && depth < 5) {
      auto fut = std::async(std::launch::async, [&, l, depth, bl] { build(l, left, depth + 1, bl); });
      build(l + 1, right, depth + 1, br);
      fut.get();
    } else {
      build(l, left, depth + 1, bl);
      build(l + 1, right, depth + 1, br);
    }
  }
};

// copy of a binary node snapshot (the vector may not grow any more at collapse time); leaves
// receive their triangle ranges in the order they are emitted
struct Collapser {
  const std::vector<BinNode>& bin;
  std::vector<Node4>& out;
  std::vector<uint32_t>& order;
  uint32_t max_depth = 0;

  uint32_t leaf_ref(const BinNode& b) {
    const uint32_t first = (uint32_t)order.size();
    if (first + b.count - 1u > kLeafFirstMask) throw std::length_error("too many triangle references for a leaf index");
    for (uint32_t i = 0; i < b.count; ++i) order.push_back(b.tri[i]);
    return kLeafBit | ((b.count - 1u) << kLeafCountShift) | (first & kLeafFirstMask);
  }

  uint32_t emit(int32_t bi, uint32_t depth) {
    max_depth = std::max(max_depth, depth);
    const uint32_t my = (uint32_t)out.size();
    out.emplace_back();
    int32_t kids[4];
    int nk = 0;
    const BinNode& b = bin[bi];
    kids[nk++] = b.left;
    kids[nk++] = b.right;
    while (nk < 4) {
      int pick = -1;
      double best = -1.0;
      for (int i = 0; i < nk; ++i) {
        const BinNode& c = bin[kids[i]];
        if (c.left < 0) continue;
        const double a = c.box.area();
        if (a > best) {
          best = a;
          pick = i;
        }
      }
      if (pick < 0) break;
      const BinNode& c = bin[kids[pick]];
      kids[pick] = c.left;
      kids[nk++] = c.right;
    }
    Node4 n;
    std::memset(&n, 0, sizeof(n));
    for (int i = 0; i < 4; ++i) {
      n.lox[i] = n.loy[i] = n.loz[i] = 1.0f;
      n.hix[i] = n.hiy[i] = n.hiz[i] = -1.0f;
      n.child[i] = kNodeEmpty;
    }
    for (int i = 0; i < nk; ++i) {
      const BinNode& c = bin[kids[i]];
      n.lox[i] = c.box.lo[0]; n.hix[i] = c.box.hi[0];
      n.loy[i] = c.box.lo[1]; n.hiy[i] = c.box.hi[1];
      n.loz[i] = c.box.lo[2]; n.hiz[i] = c.box.hi[2];
      n.child[i] = c.left < 0 ? leaf_ref(c) : 0u;
    }
    out[my] = n;
    for (int i = 0; i < nk; ++i) {
      const BinNode& c = bin[kids[i]];
      if (c.left >= 0) {
        const uint32_t ci = emit(kids[i], depth + 1);
        out[my].child[i] = ci;
      }
    }
    return my;
  }
};

}  // namespace

// Spatial splits: references they may add, as a fraction of the triangles, and the overlap of
// the best object split's children (a fraction of the scene box's area) above which they are
// tried
constexpr double kSpatialBudget = 6.0;
constexpr double kSpatialOverlap = 1e-4;

// Build from a triangle soup [n][9]; returns nodes (root at 0, always an inner node), the
// triangle index of every leaf slot (a triangle split in space fills several) and the depth of
// the 4-wide tree.
void build_bvh4(const float* tv, uint32_t n, std::vector<Node4>& nodes, std::vector<uint32_t>& order,
                uint32_t& depth) {
  nodes.clear();
  order.clear();
  if (n <= Builder::kLeafMax) {
    // an inner root with a single leaf child, so that the walk always starts at a node
    Box box;
    for (uint32_t i = 0; i < n; ++i) {
      box.grow(tv + 9 * (size_t)i);
      box.grow(tv + 9 * (size_t)i + 3);
      box.grow(tv + 9 * (size_t)i + 6);
    }
    Node4 r;
    std::memset(&r, 0, sizeof(r));
    for (int i = 0; i < 4; ++i) {
      r.lox[i] = r.loy[i] = r.loz[i] = 1.0f;
      r.hix[i] = r.hiy[i] = r.hiz[i] = -1.0f;
      r.child[i] = kNodeEmpty;
    }
    if (n > 0) {
      r.lox[0] = box.lo[0]; r.hix[0] = box.hi[0];
      r.loy[0] = box.lo[1]; r.hiy[0] = box.hi[1];
      r.loz[0] = box.lo[2]; r.hiz[0] = box.hi[2];
      r.child[0] = kLeafBit | ((n - 1u) << kLeafCountShift);
      for (uint32_t i = 0; i < n; ++i) order.push_back(i);
    }
    nodes.push_back(r);
    depth = 1;
    return;
  }
  std::vector<Ref> refs(n);
  {
    const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nth; ++w)
      th.emplace_back([&, w] {
        for (size_t i = w; i < n; i += nth) {
          Box b;
          b.grow(tv + 9 * i);
          b.grow(tv + 9 * i + 3);
          b.grow(tv + 9 * i + 6);
          refs[i] = Ref{b, (uint32_t)i};
        }
      });
    for (auto& t : th) t.join();
  }
  Box root;
  for (const Ref& r : refs) root.grow(r.box);
  Builder B;
  B.tv = tv;
  // extra references at most kSpatialBudget n, and leaf indices within 24 bits
  const int64_t budget = std::min<int64_t>((int64_t)(kSpatialBudget * n), (int64_t)kLeafFirstMask - (int64_t)n);
  B.min_overlap = kSpatialOverlap * root.area();
  B.nodes.reserve(2 * (size_t)n + 8);
  B.nodes.emplace_back();
  B.build(0, refs, 0, std::max<int64_t>(budget, 0));
  nodes.reserve(B.nodes.size() / 2 + 8);
  order.reserve(B.nodes.size() / 2 + 8);
  Collapser Cl{B.nodes, nodes, order};
  Cl.emit(0, 1);
  depth = Cl.max_depth;
}

// Solid angle, first and second direction moments of the 64 cells of the 8x8 hemi-octahedral
// atlas, in the probe's local frame (z = normal).  Each cell is integrated as two triangles
// split along the diagonal where the map |a| + |b| has its kink, with a 20-point
// Gauss-Legendre rule in each of the two collapsed coordinates on 4x4 sub-blocks.
void cell_moment_table(double out[64][10]) {
  // Gauss-Legendre nodes/weights of order 20 via Newton iteration on P_20
  const int G = 20;
  double xg[G], wg[G];
  for (int i = 0; i < G; ++i) {
    double x = std::cos(M_PI * (i + 0.75) / (G + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= G; ++k) {
        const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double dp = G * (x * p1 - p0) / (x * x - 1.0);
      const double dx = p1 / dp;
      x -= dx;
      if (std::fabs(dx) < 1e-16) break;
    }
    double p0 = 1.0, p1 = x;
    for (int k = 2; k <= G; ++k) {
      const double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    const double dp = G * (x * p1 - p0) / (x * x - 1.0);
    xg[i] = x;
    wg[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  auto tri = [&](const double* A, const double* Bv, const double* Cv, double* acc) {
    // x = A + s (B - A) + s t (C - B), s, t in [0,1], Jacobian s |det|
    const double e1[2] = {Bv[0] - A[0], Bv[1] - A[1]};
    const double e2[2] = {Cv[0] - Bv[0], Cv[1] - Bv[1]};
    const double jac = std::fabs(e1[0] * e2[1] - e1[1] * e2[0]);
    const int SUB = 4;
    for (int bs = 0; bs < SUB; ++bs)
      for (int bt = 0; bt < SUB; ++bt)
        for (int i = 0; i < G; ++i)
          for (int j = 0; j < G; ++j) {
            const double s = (bs + 0.5 * (xg[i] + 1.0)) / SUB;
            const double t = (bt + 0.5 * (xg[j] + 1.0)) / SUB;
            const double w = wg[i] * wg[j] * 0.25 / (SUB * SUB) * s * jac;
            const double u = A[0] + s * e1[0] + s * t * e2[0];
            const double v = A[1] + s * e1[1] + s * t * e2[1];
            const double a = 0.5 * (u + v), b = 0.5 * (u - v);
            const double z = 1.0 - std::fabs(a) - std::fabs(b);
            const double r2 = a * a + b * b + z * z, r = std::sqrt(r2);
            const double dw = w * 0.5 / (r2 * r);
            const double x = a / r, y = b / r, zz = z / r;
            acc[0] += dw;
            acc[1] += dw * x; acc[2] += dw * y; acc[3] += dw * zz;
            acc[4] += dw * x * x; acc[5] += dw * y * y; acc[6] += dw * zz * zz;
            acc[7] += dw * x * y; acc[8] += dw * x * zz; acc[9] += dw * y * zz;
          }
  };
  for (int iy = 0; iy < 8; ++iy)
    for (int ix = 0; ix < 8; ++ix) {
      const double u0 = -1.0 + 0.25 * ix, u1 = u0 + 0.25, v0 = -1.0 + 0.25 * iy, v1 = v0 + 0.25;
      const double p00[2] = {u0, v0}, p10[2] = {u1, v0}, p01[2] = {u0, v1}, p11[2] = {u1, v1};
      double acc[10] = {0};
      if (ix + iy == 7) {
        tri(p10, p01, p00, acc);
        tri(p10, p11, p01, acc);
      } else {
        tri(p00, p10, p11, acc);
        tri(p00, p11, p01, acc);
      }
      for (int k = 0; k < 10; ++k) out[8 * iy + ix][k] = acc[k];
    }
}

}  // namespace gi
