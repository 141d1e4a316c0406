// Host-side construction of the 4-wide BVH (binned SAH binary tree, collapsed to 4 children
// per node) and of the hemi-octahedral cell moment table.
#include "gi_host.hpp"

#include <algorithm>
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
  uint32_t first = 0, count = 0;   // leaf range in the reordered triangle index array
};

struct Builder {
  const std::vector<Box>* tri_box;
  const std::vector<float>* cen;   // [n][3]
  std::vector<uint32_t>* ids;
  std::vector<BinNode> nodes;
  std::mutex mu;

  static constexpr int kBins = 64;
  static constexpr uint32_t kLeafMax = 2;

  int32_t alloc_pair() {
    std::lock_guard<std::mutex> g(mu);
    nodes.emplace_back();
    nodes.emplace_back();
    return (int32_t)nodes.size() - 2;
  }

  // builds node `ni` over ids[first, first+count); returns nothing, fills nodes[ni]
  void build(int32_t ni, uint32_t first, uint32_t count, int depth) {
    Box box, cbox;
    for (uint32_t i = first; i < first + count; ++i) {
      const uint32_t t = (*ids)[i];
      box.grow((*tri_box)[t]);
      cbox.grow(&(*cen)[3 * (size_t)t]);
    }
    BinNode node;
    node.box = box;
    if (count <= kLeafMax) {
      node.first = first;
      node.count = count;
      std::lock_guard<std::mutex> g(mu);
      nodes[ni] = node;
      return;
    }
    // binned SAH over all three axes
    double best_cost = 1e300;
    int best_axis = -1, best_split = -1;
    for (int a = 0; a < 3; ++a) {
      const float ext = cbox.hi[a] - cbox.lo[a];
      if (!(ext > 0.0f)) continue;
      Box bb[kBins];
      uint32_t bc[kBins] = {0};
      const double k = kBins / (double)ext * (1.0 - 1e-6);
      for (uint32_t i = first; i < first + count; ++i) {
        const uint32_t t = (*ids)[i];
        int b = (int)((((*cen)[3 * (size_t)t + a]) - cbox.lo[a]) * k);
        b = std::min(std::max(b, 0), kBins - 1);
        bb[b].grow((*tri_box)[t]);
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
        if (cost < best_cost) {
          best_cost = cost;
          best_axis = a;
          best_split = b;
        }
      }
    }
    uint32_t mid;
    if (best_axis < 0) {
      mid = first + count / 2;   // all centroids coincide: split the list in half
    } else {
      const float ext = cbox.hi[best_axis] - cbox.lo[best_axis];
      const double k = kBins / (double)ext * (1.0 - 1e-6);
      auto it = std::partition(ids->begin() + first, ids->begin() + first + count, [&](uint32_t t) {
        int b = (int)((((*cen)[3 * (size_t)t + best_axis]) - cbox.lo[best_axis]) * k);
        b = std::min(std::max(b, 0), kBins - 1);
        return b < best_split;
      });
      mid = (uint32_t)(it - ids->begin());
      if (mid == first || mid == first + count) mid = first + count / 2;
    }
    const int32_t l = alloc_pair();
    node.left = l;
    node.right = l + 1;
    {
      std::lock_guard<std::mutex> g(mu);
      nodes[ni] = node;
    }
    const uint32_t nl = mid - first, nr = first + count - mid;
    if (count > 200000 && depth < 5) {
      auto fut = std::async(std::launch::async, [&, l, first, nl, depth] { build(l, first, nl, depth + 1); });
      build(l + 1, mid, nr, depth + 1);
      fut.get();
    } else {
      build(l, first, nl, depth + 1);
      build(l + 1, mid, nr, depth + 1);
    }
  }
};

// copy of a binary node snapshot (the vector may not grow any more at collapse time)
struct Collapser {
  const std::vector<BinNode>& bin;
  std::vector<Node4>& out;
  uint32_t max_depth = 0;

  uint32_t leaf_ref(const BinNode& b) const {
    return kLeafBit | ((b.count - 1u) << kLeafCountShift) | (b.first & kLeafFirstMask);
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

// Build from a triangle soup [n][9]; returns nodes (root at 0, always an inner node), the
// leaf order of the triangles and the depth of the 4-wide tree.
void build_bvh4(const float* tv, uint32_t n, std::vector<Node4>& nodes, std::vector<uint32_t>& order,
                uint32_t& depth) {
  std::vector<Box> tri_box(n);
  std::vector<float> cen(3 * (size_t)n);
  const unsigned nth = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  {
    std::vector<std::thread> th;
    for (unsigned w = 0; w < nth; ++w)
      th.emplace_back([&, w] {
        for (size_t i = w; i < n; i += nth) {
          const float* v = tv + 9 * i;
          Box b;
          b.grow(v);
          b.grow(v + 3);
          b.grow(v + 6);
          tri_box[i] = b;
          for (int a = 0; a < 3; ++a) cen[3 * i + a] = (b.lo[a] + b.hi[a]) * 0.5f;
        }
      });
    for (auto& t : th) t.join();
  }
  order.resize(n);
  std::iota(order.begin(), order.end(), 0u);
  Builder B;
  B.tri_box = &tri_box;
  B.cen = &cen;
  B.ids = &order;
  B.nodes.reserve(2 * (size_t)n + 8);
  B.nodes.emplace_back();
  if (n <= Builder::kLeafMax) {
    // force an inner root with a single leaf child so the walk always starts at a node
    Box box;
    for (uint32_t i = 0; i < n; ++i) box.grow(tri_box[i]);
    BinNode leaf;
    leaf.box = box;
    leaf.first = 0;
    leaf.count = n;
    BinNode empty;
    empty.first = 0;
    empty.count = 0;
    B.nodes[0].box = box;
    B.nodes.push_back(leaf);
    B.nodes[0].left = 1;
    B.nodes[0].right = -1;
    nodes.clear();
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
    }
    nodes.push_back(r);
    depth = 1;
    return;
  }
  B.build(0, 0, n, 0);
  nodes.clear();
  nodes.reserve(B.nodes.size() / 2 + 8);
  Collapser Cl{B.nodes, nodes};
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
