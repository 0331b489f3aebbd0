// Host-side mesh preparation: validation, shell topology, SAH BVH.
//
//  * validation -- every facet edge is shared with exactly one other facet of
//    the same region traversed in the opposite direction (closed, consistently
//    wound 2-manifold shells), every shell has positive signed volume (outward
//    Eq. 5 normals), and no two shells intersect or come closer than the
//    minimum gap (coincident surfaces must be separated inside-out,
//    Sec. 2.4.2, Fig. 6);
//  * topology -- the region outside each shell is found with the ray-parity
//    rule of Sec. 2.4.2 from a point on the shell, in FP64, so the per-facet
//    inner/outer pair of the Triangle structure (Sec. 2.2.3) is derived rather
//    than declared;
//  * BVH -- binned surface-area-heuristic build, flattened depth-first into
//    64-byte two-child nodes, facets reordered into 48-byte leaf records.
#include <math.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <numeric>
#include <thread>
#include <unordered_map>

#include "gadep.h"
#include "gadep_internal.h"

namespace gadep {
namespace {

struct D3 {
  double x, y, z;
};
inline D3 operator-(D3 a, D3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline D3 operator+(D3 a, D3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline D3 operator*(double s, D3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dot(D3 a, D3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline D3 cross(D3 a, D3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double len(D3 a) { return sqrt(dot(a, a)); }
inline double clamp01(double x) { return x < 0 ? 0 : (x > 1 ? 1 : x); }

// Host threads for the heavy loops of the preparation (up to 16).
int worker_count(int64_t items) {
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int64_t by_size = items / 4096 + 1;
  return static_cast<int>(std::min<int64_t>(std::min<unsigned>(hw, 16u), by_size));
}

template <class F>
void run_workers(int n, F&& work) {
  std::vector<std::thread> th;
  for (int w = 1; w < n; ++w) th.emplace_back(work, w);
  work(0);
  for (auto& t : th) t.join();
}

struct Box {
  float lo[3], hi[3];
  void reset() {
    for (int a = 0; a < 3; ++a) {
      lo[a] = INFINITY;
      hi[a] = -INFINITY;
    }
  }
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

struct Ref {
  Box box;
  float c[3];
  int32_t id;
};

// ---------------------------------------------------------------------------
// BVH build

class Builder {
 public:
  Builder(std::vector<Ref>& refs, int method) : refs_(refs), method_(method) {}

  void run(std::vector<BvhNode>& nodes, int32_t& depth, double& sah) {
    nodes_.clear();
    max_depth_ = 0;
    const int64_t n = static_cast<int64_t>(refs_.size());
    Box all;
    nodes_.emplace_back();  // root
    if (n <= kLeafMax) {
      all.reset();
      for (auto& r : refs_) all.grow(r.box);
      Box empty;
      empty.reset();
      set_node(0, all, leaf_code(0, static_cast<int32_t>(n)), empty, leaf_code(0, 0));
      max_depth_ = 1;
    } else {
      build_into(0, 0, n, 1, all);
    }
    nodes.swap(nodes_);
    depth = max_depth_;
    sah = sah_cost(nodes, all);
  }

 private:
  std::vector<Ref>& refs_;
  int method_;
  std::vector<BvhNode> nodes_;
  int32_t max_depth_ = 0;
  static constexpr int kBins = 32;

  void set_node(int32_t idx, const Box& l, int32_t lc, const Box& r, int32_t rc) {
    BvhNode& nd = nodes_[idx];
    for (int a = 0; a < 3; ++a) {
      nd.lmin[a] = l.lo[a];
      nd.lmax[a] = l.hi[a];
      nd.rmin[a] = r.lo[a];
      nd.rmax[a] = r.hi[a];
    }
    nd.child[0] = lc;
    nd.child[1] = rc;
    nd.pad[0] = nd.pad[1] = 0;
  }

  // Splits refs[b, e) (more than kLeafMax of them) under node `idx`.
  void build_into(int32_t idx, int64_t b, int64_t e, int depth, Box& box_out) {
    max_depth_ = std::max(max_depth_, depth);
    int64_t mid = split(b, e, depth);
    Box lb, rb;
    int32_t lc = subtree(b, mid, depth, lb);
    int32_t rc = subtree(mid, e, depth, rb);
    set_node(idx, lb, lc, rb, rc);
    box_out = lb;
    box_out.grow(rb);
  }

  int32_t subtree(int64_t b, int64_t e, int depth, Box& box) {
    const int64_t n = e - b;
    if (n <= kLeafMax) {
      box.reset();
      for (int64_t i = b; i < e; ++i) box.grow(refs_[i].box);
      // a small set stays a leaf unless splitting it is cheaper by the SAH
      int64_t mid = -1;
      if (n < 2 || method_ != 0 || depth >= kMaxDepth - 1 ||
          best_split(b, e, &mid) >= kCostIsect * n * box.area())
        return leaf_code(b, static_cast<int32_t>(n));
    }
    int32_t idx = static_cast<int32_t>(nodes_.size());
    nodes_.emplace_back();
    build_into(idx, b, e, depth + 1, box);
    return idx;
  }

  static constexpr double kCostTrav = 1.2;   // one node visit (two box tests)
  static constexpr double kCostIsect = 1.0;  // one facet test

  // Cheapest SAH split of refs[b, e): centroid bins along each axis, plus a
  // split of large boxes from small ones (needed when large facets, such as
  // the faces of a world box, share centroid coordinates with small ones).
  // Partitions refs and sets *mid on success; returns the SAH cost or +inf.
  double best_split(int64_t b, int64_t e, int64_t* mid) {
    Box cb, all;
    cb.reset();
    all.reset();
    for (int64_t i = b; i < e; ++i) {
      cb.grow(refs_[i].c);
      all.grow(refs_[i].box);
    }
    const double area = all.area();
    double best = INFINITY;
    int best_kind = -1, best_bin = -1;  // kind 0..2: centroid axis; 3: box size
    float best_lo = 0, best_scale = 0;
    auto value = [](const Ref& r, int kind) {
      return kind < 3 ? r.c[kind] : logf(static_cast<float>(r.box.area()) + 1e-30f);
    };
    auto key = [&](const Ref& r, int kind, float lo, float scale) {
      return std::min(kBins - 1, std::max(0, static_cast<int>((value(r, kind) - lo) * scale)));
    };
    for (int kind = 0; kind < 4; ++kind) {
      float lo = INFINITY, hi = -INFINITY;
      for (int64_t i = b; i < e; ++i) {
        const float v = value(refs_[i], kind);
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
      const float ext = hi - lo;
      if (!(ext > 0)) continue;
      const float scale = kBins * (1.0f - 1e-6f) / ext;
      Box bins[kBins];
      int64_t cnt[kBins] = {0};
      for (auto& bx : bins) bx.reset();
      for (int64_t i = b; i < e; ++i) {
        const int k = key(refs_[i], kind, lo, scale);
        cnt[k]++;
        bins[k].grow(refs_[i].box);
      }
      double right_area[kBins];
      int64_t right_cnt[kBins];
      Box acc;
      acc.reset();
      int64_t c = 0;
      for (int k = kBins - 1; k > 0; --k) {
        acc.grow(bins[k]);
        c += cnt[k];
        right_area[k] = acc.area();
        right_cnt[k] = c;
      }
      acc.reset();
      c = 0;
      for (int k = 0; k < kBins - 1; ++k) {
        acc.grow(bins[k]);
        c += cnt[k];
        if (c == 0 || right_cnt[k + 1] == 0) continue;
        const double cost = kCostTrav * area +
                            kCostIsect * (acc.area() * c + right_area[k + 1] * right_cnt[k + 1]);
        if (cost < best) {
          best = cost;
          best_kind = kind;
          best_bin = k;
          best_lo = lo;
          best_scale = scale;
        }
      }
    }
    if (best_kind < 0) return INFINITY;
    auto it = std::partition(refs_.begin() + b, refs_.begin() + e, [&](const Ref& r) {
      return key(r, best_kind, best_lo, best_scale) <= best_bin;
    });
    const int64_t m = it - refs_.begin();
    if (m <= b || m >= e) return INFINITY;
    *mid = m;
    return best;
  }

  int64_t split(int64_t b, int64_t e, int depth) {
    int64_t mid = -1;
    if (method_ == 0 && depth < kMaxDepth - 16 && best_split(b, e, &mid) < INFINITY) return mid;
    // object median along the widest centroid extent
    Box cb;
    cb.reset();
    for (int64_t i = b; i < e; ++i) cb.grow(refs_[i].c);
    int a = 0;
    for (int k = 1; k < 3; ++k)
      if (cb.hi[k] - cb.lo[k] > cb.hi[a] - cb.lo[a]) a = k;
    mid = b + (e - b) / 2;
    std::nth_element(refs_.begin() + b, refs_.begin() + mid, refs_.begin() + e,
                     [a](const Ref& x, const Ref& y) {
                       return x.c[a] < y.c[a] || (x.c[a] == y.c[a] && x.id < y.id);
                     });
    return mid;
  }

  static double box_area(const float* lo, const float* hi) {
    Box b;
    for (int a = 0; a < 3; ++a) {
      b.lo[a] = lo[a];
      b.hi[a] = hi[a];
    }
    return b.area();
  }

  // SAH cost, unit cost per node visit and per facet test, relative to the root
  static double sah_cost(const std::vector<BvhNode>& nodes, const Box& root) {
    double ra = root.area();
    if (!(ra > 0)) return 0.0;
    double cost = 1.0;  // root visit
    for (const BvhNode& nd : nodes) {
      const float* lo[2] = {nd.lmin, nd.rmin};
      const float* hi[2] = {nd.lmax, nd.rmax};
      for (int c = 0; c < 2; ++c) {
        double a = box_area(lo[c], hi[c]) / ra;
        if (nd.child[c] >= 0)
          cost += a;
        else
          cost += a * ((~nd.child[c]) & 7);
      }
    }
    return cost;
  }
};

// ---------------------------------------------------------------------------
// Transport BVH with spatial splits (Stich, Friedrich and Dietrich, HPG 2009).
//
// Long, thin facets -- fan caps, full-height side walls -- have boxes far
// larger than themselves, and no partition of whole facets separates them.
// Besides the object partitions above, each node here also tries to split
// space: a facet that straddles the plane is referenced from both sides, each
// reference keeping only the box of the facet's part on its side, so a facet
// may be listed in several leaves.  That is harmless for closest-hit search;
// crossing-parity counts use the plain BVH instead.

double nodes_sah(const std::vector<BvhNode>& nodes, double root_area) {
  if (!(root_area > 0)) return 0.0;
  double cost = 1.0;  // root visit
  for (const BvhNode& nd : nodes) {
    const float* lo[2] = {nd.lmin, nd.rmin};
    const float* hi[2] = {nd.lmax, nd.rmax};
    for (int c = 0; c < 2; ++c) {
      Box b;
      for (int a = 0; a < 3; ++a) {
        b.lo[a] = lo[c][a];
        b.hi[a] = hi[c][a];
      }
      const double f = b.area() / root_area;
      cost += nd.child[c] >= 0 ? f : f * ((~nd.child[c]) & 7);
    }
  }
  return cost;
}

class SplitBuilder {
 public:
  SplitBuilder(const float* xyz, const int32_t* tv, int64_t max_refs, bool cut_pieces = false)
      : xyz_(xyz), tv_(tv), max_refs_(max_refs), cut_pieces_(cut_pieces) {}

  // refs: one whole-facet reference per facet.  ids receives the facet of
  // each reference slot in leaf order.  With a budget for extra references
  // (max_refs above the facet count), long, thin facets are cut into pieces
  // first when cut_pieces is set (these do not count against the budget),
  // then spatial splits use it.
  void run(std::vector<Ref> refs, std::vector<BvhNode>& nodes, std::vector<int32_t>& ids,
           int32_t& depth, double& sah) {
    nodes_.clear();
    ids_.clear();
    max_depth_ = 1;
    if (cut_pieces_ && max_refs_ > static_cast<int64_t>(refs.size())) presplit(refs);
    n_refs_ = static_cast<int64_t>(refs.size());
    Box all;
    all.reset();
    for (const Ref& r : refs) all.grow(r.box);
    root_area_ = all.area();
    nodes_.emplace_back();
    if (static_cast<int>(refs.size()) <= kSplitLeafMax) {
      Box empty;
      empty.reset();
      const int32_t code = emit_leaf(refs);
      set_node(0, all, code, empty, leaf_code(static_cast<int64_t>(ids_.size()), 0));
    } else {
      Box b;
      build(0, std::move(refs), all, 1, b);
    }
    nodes.swap(nodes_);
    ids.swap(ids_);
    depth = max_depth_;
    sah = nodes_sah(nodes, root_area_);
  }

 private:
  const float* xyz_;
  const int32_t* tv_;
  int64_t max_refs_;
  bool cut_pieces_ = false;
  int64_t n_refs_ = 0;
  double root_area_ = 0.0;
  std::vector<BvhNode> nodes_;
  std::vector<int32_t> ids_;
  int32_t max_depth_ = 0;
  static constexpr int kBins = 32;
  // a node visit priced at two facet tests: the transport kernel runs the
  // node and facet steps of a wavefront's lanes one after the other in each
  // iteration, and fewer, fuller leaves measured faster than the textbook 1.2
  static constexpr double kCostTrav = 2.0;
  static constexpr double kCostIsect = 1.0;
  static constexpr double kMinOverlap = 1e-5;  // spatial splits only where children overlap
  static constexpr int kSplitLeafMax = kLeafMax;
  // early split clipping of long, thin facets (Ernst and Greiner 2007): a
  // reference is cut in half across its longest box side until that side is
  // at most kPieceWidths facet widths (twice the area over the longest edge)
  // or the facet has kMaxPieces pieces.  The fan caps of the detector shells
  // are the case in point: their wedges' boxes overlap near the centre, and a
  // segment that starts on one of them would otherwise visit most of them.
  static constexpr double kPieceWidths = 8.0;
  static constexpr int kMaxPieces = 32;

 public:
  // Meshes below this many facets keep whole facets: their BVHs stay small
  // enough to live in cache, and several of them (one per job of a batch)
  // may share it, so pieces would cost more in footprint than they save.
  static constexpr int64_t kPieceMinFacets = 4096;

 private:

  void presplit(std::vector<Ref>& refs) {
    std::vector<Ref> out;
    out.reserve(refs.size());
    std::vector<Ref> st;
    for (const Ref& r : refs) {
      const float* v[3] = {xyz_ + 3 * tv_[3 * r.id], xyz_ + 3 * tv_[3 * r.id + 1],
                           xyz_ + 3 * tv_[3 * r.id + 2]};
      double e[3][3];
      double lmax = 0;
      for (int i = 0; i < 3; ++i) {
        for (int k = 0; k < 3; ++k) e[i][k] = static_cast<double>(v[(i + 1) % 3][k]) - v[i][k];
        lmax = std::max(lmax, sqrt(e[i][0] * e[i][0] + e[i][1] * e[i][1] + e[i][2] * e[i][2]));
      }
      const double cx = e[0][1] * e[1][2] - e[0][2] * e[1][1];
      const double cy = e[0][2] * e[1][0] - e[0][0] * e[1][2];
      const double cz = e[0][0] * e[1][1] - e[0][1] * e[1][0];
      const double cap = kPieceWidths * sqrt(cx * cx + cy * cy + cz * cz) / std::max(lmax, 1e-30);
      st.assign(1, r);
      int pieces = 1;
      while (!st.empty()) {
        Ref p = st.back();
        st.pop_back();
        int ax = 0;
        for (int a = 1; a < 3; ++a)
          if (p.box.hi[a] - p.box.lo[a] > p.box.hi[ax] - p.box.lo[ax]) ax = a;
        Box L, R;
        if (p.box.hi[ax] - p.box.lo[ax] > cap && pieces < kMaxPieces)
          split_ref(p, ax, 0.5f * (p.box.lo[ax] + p.box.hi[ax]), L, R);
        else
          L.reset();
        if (!valid(L) || !valid(R)) {
          out.push_back(p);
          continue;
        }
        Ref a = p, b = p;
        a.box = L;
        b.box = R;
        for (int k = 0; k < 3; ++k) {
          a.c[k] = 0.5f * (L.lo[k] + L.hi[k]);
          b.c[k] = 0.5f * (R.lo[k] + R.hi[k]);
        }
        st.push_back(a);
        st.push_back(b);
        ++pieces;
      }
    }
    // the pieces do not use up the spatial-split budget
    max_refs_ += static_cast<int64_t>(out.size()) - static_cast<int64_t>(refs.size());
    refs.swap(out);
  }

  struct Plan {
    double cost = INFINITY;
    int kind = -1;  // 0..2 centroid axis, 3 box size, 4 spatial
    int axis = 0, bin = 0;
    float lo = 0, scale = 0, pos = 0;
    Box left, right;  // spatial: child boxes and reference counts from the bins
    int64_t n_left = 0, n_right = 0;
  };

  void set_node(int32_t idx, const Box& l, int32_t lc, const Box& r, int32_t rc) {
    BvhNode& nd = nodes_[idx];
    for (int a = 0; a < 3; ++a) {
      nd.lmin[a] = l.lo[a];
      nd.lmax[a] = l.hi[a];
      nd.rmin[a] = r.lo[a];
      nd.rmax[a] = r.hi[a];
    }
    nd.child[0] = lc;
    nd.child[1] = rc;
    nd.pad[0] = nd.pad[1] = 0;
  }

  int32_t emit_leaf(const std::vector<Ref>& refs) {
    // a facet cut into pieces is listed once per leaf
    const int64_t first = static_cast<int64_t>(ids_.size());
    for (const Ref& r : refs)
      if (std::find(ids_.begin() + first, ids_.end(), r.id) == ids_.end()) ids_.push_back(r.id);
    return leaf_code(first, static_cast<int32_t>(static_cast<int64_t>(ids_.size()) - first));
  }

  static Box bounds(const std::vector<Ref>& refs) {
    Box b;
    b.reset();
    for (const Ref& r : refs) b.grow(r.box);
    return b;
  }

  static void widen(Box& b) {
    // one part in 2^22 outward, so rounding of the clipped corners never
    // uncovers a sliver of the facet
    for (int a = 0; a < 3; ++a) {
      const float m = 2.4e-7f * std::max(fabsf(b.lo[a]), fabsf(b.hi[a])) + 1e-30f;
      b.lo[a] -= m;
      b.hi[a] += m;
    }
  }

  // boxes of the parts of reference r on either side of the plane x[axis] = pos
  void split_ref(const Ref& r, int axis, float pos, Box& L, Box& R) const {
    L.reset();
    R.reset();
    const float* v[3] = {xyz_ + 3 * tv_[3 * r.id], xyz_ + 3 * tv_[3 * r.id + 1],
                         xyz_ + 3 * tv_[3 * r.id + 2]};
    for (int i = 0; i < 3; ++i) {
      const float* p = v[i];
      const float* q = v[(i + 1) % 3];
      if (p[axis] <= pos) L.grow(p);
      if (p[axis] >= pos) R.grow(p);
      if ((p[axis] < pos && pos < q[axis]) || (p[axis] > pos && pos > q[axis])) {
        const double t = (static_cast<double>(pos) - p[axis]) / (static_cast<double>(q[axis]) - p[axis]);
        float x[3];
        for (int k = 0; k < 3; ++k) x[k] = static_cast<float>(p[k] + t * (static_cast<double>(q[k]) - p[k]));
        x[axis] = pos;
        L.grow(x);
        R.grow(x);
      }
    }
    widen(L);
    widen(R);
    for (int a = 0; a < 3; ++a) {
      L.lo[a] = std::max(L.lo[a], r.box.lo[a]);
      L.hi[a] = std::min(L.hi[a], r.box.hi[a]);
      R.lo[a] = std::max(R.lo[a], r.box.lo[a]);
      R.hi[a] = std::min(R.hi[a], r.box.hi[a]);
    }
    L.hi[axis] = std::min(L.hi[axis], pos);
    R.lo[axis] = std::max(R.lo[axis], pos);
  }

  static bool valid(const Box& b) {
    return b.lo[0] <= b.hi[0] && b.lo[1] <= b.hi[1] && b.lo[2] <= b.hi[2];
  }

  static Box overlap(const Box& a, const Box& b) {
    Box o;
    for (int k = 0; k < 3; ++k) {
      o.lo[k] = std::max(a.lo[k], b.lo[k]);
      o.hi[k] = std::min(a.hi[k], b.hi[k]);
    }
    return o;
  }

  static float centroid_value(const Ref& r, int kind) {
    return kind < 3 ? 0.5f * (r.box.lo[kind] + r.box.hi[kind])
                    : logf(static_cast<float>(r.box.area()) + 1e-30f);
  }

  static int key(const Ref& r, int kind, float lo, float scale) {
    return std::min(kBins - 1, std::max(0, static_cast<int>((centroid_value(r, kind) - lo) * scale)));
  }

  // best partition of whole references (centroid bins on three axes, box size)
  void object_plan(const std::vector<Ref>& refs, double area, Plan& best, Box* lbox, Box* rbox) const {
    for (int kind = 0; kind < 4; ++kind) {
      float lo = INFINITY, hi = -INFINITY;
      for (const Ref& r : refs) {
        const float v = centroid_value(r, kind);
        lo = std::min(lo, v);
        hi = std::max(hi, v);
      }
      if (!(hi - lo > 0)) continue;
      const float scale = kBins * (1.0f - 1e-6f) / (hi - lo);
      Box bins[kBins];
      int64_t cnt[kBins] = {0};
      for (Box& b : bins) b.reset();
      for (const Ref& r : refs) {
        const int k = key(r, kind, lo, scale);
        cnt[k]++;
        bins[k].grow(r.box);
      }
      Box rb[kBins];
      int64_t rc[kBins];
      Box acc;
      acc.reset();
      int64_t c = 0;
      for (int k = kBins - 1; k > 0; --k) {
        acc.grow(bins[k]);
        c += cnt[k];
        rb[k] = acc;
        rc[k] = c;
      }
      acc.reset();
      c = 0;
      for (int k = 0; k < kBins - 1; ++k) {
        acc.grow(bins[k]);
        c += cnt[k];
        if (c == 0 || rc[k + 1] == 0) continue;
        const double cost = kCostTrav * area + kCostIsect * (acc.area() * c + rb[k + 1].area() * rc[k + 1]);
        if (cost < best.cost) {
          best.cost = cost;
          best.kind = kind;
          best.bin = k;
          best.lo = lo;
          best.scale = scale;
          if (lbox) *lbox = acc;
          if (rbox) *rbox = rb[k + 1];
        }
      }
    }
  }

  // best plane splitting space (references straddling it are clipped)
  void spatial_plan(const std::vector<Ref>& refs, const Box& node, double area, Plan& best) const {
    for (int axis = 0; axis < 3; ++axis) {
      const float lo = node.lo[axis], ext = node.hi[axis] - node.lo[axis];
      if (!(ext > 0)) continue;
      const float w = ext / kBins;
      auto bin_of = [&](float x) {
        return std::min(kBins - 1, std::max(0, static_cast<int>((x - lo) / w)));
      };
      Box bins[kBins];
      int64_t enter[kBins] = {0}, leave[kBins] = {0};
      for (Box& b : bins) b.reset();
      for (const Ref& r : refs) {
        const int b0 = bin_of(r.box.lo[axis]), b1 = bin_of(r.box.hi[axis]);
        enter[b0]++;
        leave[b1]++;
        Ref cur = r;
        for (int b = b0; b < b1; ++b) {
          Box L, R;
          split_ref(cur, axis, lo + (b + 1) * w, L, R);
          if (valid(L)) bins[b].grow(L);
          if (!valid(R)) break;
          cur.box = R;
        }
        if (valid(cur.box)) bins[b1].grow(cur.box);
      }
      Box rb[kBins];
      int64_t rc[kBins];
      Box acc;
      acc.reset();
      int64_t c = 0;
      for (int k = kBins - 1; k > 0; --k) {
        acc.grow(bins[k]);
        c += leave[k];
        rb[k] = acc;
        rc[k] = c;
      }
      acc.reset();
      c = 0;
      for (int k = 0; k < kBins - 1; ++k) {
        acc.grow(bins[k]);
        c += enter[k];
        if (c == 0 || rc[k + 1] == 0) continue;
        const double la = acc.area(), ra = rb[k + 1].area();
        const double cost = kCostTrav * area + kCostIsect * (la * c + ra * rc[k + 1]);
        if (cost < best.cost) {
          best.cost = cost;
          best.kind = 4;
          best.axis = axis;
          best.pos = lo + (k + 1) * w;
          best.left = acc;
          best.right = rb[k + 1];
          best.n_left = c;
          best.n_right = rc[k + 1];
        }
      }
    }
  }

  bool apply(const std::vector<Ref>& refs, const Plan& p, std::vector<Ref>& left,
             std::vector<Ref>& right) const {
    left.clear();
    right.clear();
    if (p.kind < 4) {
      for (const Ref& r : refs) (key(r, p.kind, p.lo, p.scale) <= p.bin ? left : right).push_back(r);
    } else {
      const double al = p.left.area(), ar = p.right.area();
      const double nl = static_cast<double>(p.n_left), nr = static_cast<double>(p.n_right);
      for (const Ref& r : refs) {
        if (r.box.hi[p.axis] <= p.pos) {
          left.push_back(r);
          continue;
        }
        if (r.box.lo[p.axis] >= p.pos) {
          right.push_back(r);
          continue;
        }
        Box L, R;
        split_ref(r, p.axis, p.pos, L, R);
        // keep the whole reference on one side when that is cheaper
        Box lu = p.left, ru = p.right;
        lu.grow(r.box);
        ru.grow(r.box);
        const double c_split = al * nl + ar * nr;
        const double c_left = lu.area() * nl + ar * (nr - 1);
        const double c_right = al * (nl - 1) + ru.area() * nr;
        if (!valid(R) || (valid(L) && c_left < c_split && c_left <= c_right)) {
          left.push_back(r);
        } else if (!valid(L) || c_right < c_split) {
          right.push_back(r);
        } else {
          Ref a = r, b = r;
          a.box = L;
          b.box = R;
          left.push_back(a);
          right.push_back(b);
        }
      }
    }
    return !left.empty() && !right.empty() && left.size() < refs.size() &&
           right.size() < refs.size();
  }

  void median(const std::vector<Ref>& refs, std::vector<Ref>& left, std::vector<Ref>& right) const {
    Box cb;
    cb.reset();
    for (const Ref& r : refs) {
      float c[3];
      for (int a = 0; a < 3; ++a) c[a] = 0.5f * (r.box.lo[a] + r.box.hi[a]);
      cb.grow(c);
    }
    int a = 0;
    for (int k = 1; k < 3; ++k)
      if (cb.hi[k] - cb.lo[k] > cb.hi[a] - cb.lo[a]) a = k;
    std::vector<Ref> s = refs;
    const size_t mid = s.size() / 2;
    std::nth_element(s.begin(), s.begin() + mid, s.end(), [a](const Ref& x, const Ref& y) {
      const float cx = x.box.lo[a] + x.box.hi[a], cy = y.box.lo[a] + y.box.hi[a];
      return cx < cy || (cx == cy && x.id < y.id);
    });
    left.assign(s.begin(), s.begin() + mid);
    right.assign(s.begin() + mid, s.end());
  }

  static constexpr int64_t kParallelRefs = 65536;  // subtrees this large are built
  static constexpr int kParallelDepth = 4;          // by a thread of their own

  // splits refs (more than kSplitLeafMax, or cheaper split) under node idx
  void build(int32_t idx, std::vector<Ref> refs, const Box& box, int depth, Box& box_out) {
    max_depth_ = std::max(max_depth_, depth);
    std::vector<Ref> left, right;
    choose(refs, box, depth, left, right);
    refs.clear();
    refs.shrink_to_fit();
    Box lb = bounds(left), rb = bounds(right);
    int32_t lc, rc;
    const int64_t nl = static_cast<int64_t>(left.size()), nr = static_cast<int64_t>(right.size());
    if (nl + nr >= kParallelRefs && depth <= kParallelDepth) {
      // the right subtree goes to a builder of its own, in another thread,
      // with its share of the remaining reference budget (the split of work
      // depends only on sizes, so the result does not depend on timing)
      const int64_t spare = std::max<int64_t>(0, max_refs_ - n_refs_);
      const int64_t spare_r = spare * nr / (nl + nr);
      SplitBuilder sub(xyz_, tv_, nr + spare_r);
      sub.root_area_ = root_area_;
      sub.n_refs_ = nr;
      n_refs_ -= nr;
      max_refs_ -= nr + spare_r;
      int32_t rc_sub = 0;
      std::thread t([&]() { rc_sub = sub.child(std::move(right), rb, depth); });
      lc = child(std::move(left), lb, depth);
      t.join();
      const int32_t node_off = static_cast<int32_t>(nodes_.size());
      const int64_t id_off = static_cast<int64_t>(ids_.size());
      auto relocate = [&](int32_t c) {
        if (c >= 0) return c + node_off;
        const int32_t x = ~c;
        return leaf_code((x >> 3) + id_off, x & 7);
      };
      for (BvhNode nd : sub.nodes_) {
        nd.child[0] = relocate(nd.child[0]);
        nd.child[1] = relocate(nd.child[1]);
        nodes_.push_back(nd);
      }
      ids_.insert(ids_.end(), sub.ids_.begin(), sub.ids_.end());
      rc = relocate(rc_sub);
      n_refs_ += sub.n_refs_;
      max_refs_ += sub.max_refs_;
      max_depth_ = std::max(max_depth_, sub.max_depth_);
    } else {
      lc = child(std::move(left), lb, depth);
      rc = child(std::move(right), rb, depth);
    }
    set_node(idx, lb, lc, rb, rc);
    box_out = lb;
    box_out.grow(rb);
  }

  void choose(const std::vector<Ref>& refs, const Box& box, int depth, std::vector<Ref>& left,
              std::vector<Ref>& right) {
    if (depth < kMaxDepth - 16) {
      const double area = box.area();
      Plan obj;
      Box ol, orb;
      object_plan(refs, area, obj, &ol, &orb);
      Plan best = obj;
      if (n_refs_ < max_refs_ && obj.kind >= 0) {
        const Box ov = overlap(ol, orb);
        if (valid(ov) && ov.area() > kMinOverlap * root_area_) spatial_plan(refs, box, area, best);
      } else if (n_refs_ < max_refs_ && obj.kind < 0) {
        spatial_plan(refs, box, area, best);
      }
      if (best.kind >= 0 && apply(refs, best, left, right)) {
        n_refs_ += static_cast<int64_t>(left.size() + right.size()) - static_cast<int64_t>(refs.size());
        return;
      }
      if (obj.kind >= 0 && best.kind == 4 && apply(refs, obj, left, right)) return;
    }
    median(refs, left, right);
  }

  int32_t child(std::vector<Ref> refs, const Box& box, int depth) {
    const int64_t n = static_cast<int64_t>(refs.size());
    if (n <= kSplitLeafMax) {
      bool leaf = n < 2 || depth >= kMaxDepth - 1;
      if (!leaf) {
        Plan p;
        object_plan(refs, box.area(), p, nullptr, nullptr);
        leaf = p.cost >= kCostIsect * n * box.area();
      }
      if (leaf) return emit_leaf(refs);
    }
    const int32_t idx = static_cast<int32_t>(nodes_.size());
    nodes_.emplace_back();
    Box b;
    build(idx, std::move(refs), box, depth + 1, b);
    return idx;
  }
};

// ---------------------------------------------------------------------------
// FP64 queries over the flattened BVH (host preparation only)

class HostQuery {
 public:
  HostQuery(const std::vector<BvhNode>& nodes, const std::vector<int32_t>& order, double margin)
      : nodes_(nodes), order_(order), m_(margin) {}

  template <class F>
  void ray_all(D3 o, D3 d, F&& visit) const {
    int32_t stack[kMaxDepth + 4];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
      const BvhNode& nd = nodes_[stack[--sp]];
      const float* lo[2] = {nd.lmin, nd.rmin};
      const float* hi[2] = {nd.lmax, nd.rmax};
      for (int c = 0; c < 2; ++c) {
        if (!ray_box(o, d, lo[c], hi[c])) continue;
        int32_t ch = nd.child[c];
        if (ch >= 0) {
          stack[sp++] = ch;
        } else {
          int32_t x = ~ch;
          for (int32_t i = x >> 3, n = x & 7, k = 0; k < n; ++k) visit(order_[i + k]);
        }
      }
    }
  }

  template <class F>
  void box_all(const double* lo, const double* hi, F&& visit) const {
    int32_t stack[kMaxDepth + 4];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
      const BvhNode& nd = nodes_[stack[--sp]];
      const float* blo[2] = {nd.lmin, nd.rmin};
      const float* bhi[2] = {nd.lmax, nd.rmax};
      for (int c = 0; c < 2; ++c) {
        bool ov = true;
        for (int a = 0; a < 3 && ov; ++a)
          ov = !(hi[a] < blo[c][a] - m_ || lo[a] > bhi[c][a] + m_);
        if (!ov) continue;
        int32_t ch = nd.child[c];
        if (ch >= 0) {
          stack[sp++] = ch;
        } else {
          int32_t x = ~ch;
          for (int32_t i = x >> 3, n = x & 7, k = 0; k < n; ++k) visit(order_[i + k]);
        }
      }
    }
  }

 private:
  const std::vector<BvhNode>& nodes_;
  const std::vector<int32_t>& order_;
  double m_;

  bool ray_box(D3 o, D3 d, const float* lo, const float* hi) const {
    double t0 = 0.0, t1 = INFINITY;
    const double oo[3] = {o.x, o.y, o.z}, dd[3] = {d.x, d.y, d.z};
    for (int a = 0; a < 3; ++a) {
      double l = lo[a] - m_, h = hi[a] + m_;
      if (dd[a] == 0.0) {
        if (oo[a] < l || oo[a] > h) return false;
        continue;
      }
      double ta = (l - oo[a]) / dd[a], tb = (h - oo[a]) / dd[a];
      if (ta > tb) std::swap(ta, tb);
      t0 = std::max(t0, ta);
      t1 = std::min(t1, tb);
      if (t0 > t1) return false;
    }
    return true;
  }
};

// ---------------------------------------------------------------------------
// exact-ish FP64 facet geometry for validation

struct Tri3 {
  D3 a, b, c;
};

// crossing of segment p + s (q - p), s in [0, 1], with the facet (inclusive)
bool segment_hits(D3 p, D3 q, const Tri3& t) {
  D3 d = q - p;
  D3 e1 = t.b - t.a, e2 = t.c - t.a;
  D3 h = cross(d, e2);
  double det = dot(e1, h);
  double scale = len(e1) * len(e2) * len(d);
  if (fabs(det) <= 1e-15 * scale) return false;  // parallel: covered by distances
  double inv = 1.0 / det;
  D3 s = p - t.a;
  double u = dot(s, h) * inv;
  if (u < 0 || u > 1) return false;
  D3 qv = cross(s, e1);
  double v = dot(d, qv) * inv;
  if (v < 0 || u + v > 1) return false;
  double w = dot(e2, qv) * inv;
  return w >= 0 && w <= 1;
}

// distance from p to the closest point of the facet (Voronoi-region walk)
double point_tri_dist(D3 p, const Tri3& t) {
  D3 ab = t.b - t.a, ac = t.c - t.a, ap = p - t.a;
  double d1 = dot(ab, ap), d2 = dot(ac, ap);
  if (d1 <= 0 && d2 <= 0) return len(p - t.a);
  D3 bp = p - t.b;
  double d3 = dot(ab, bp), d4 = dot(ac, bp);
  if (d3 >= 0 && d4 <= d3) return len(p - t.b);
  double vc = d1 * d4 - d3 * d2;
  if (vc <= 0 && d1 >= 0 && d3 <= 0) {
    double s = d1 / (d1 - d3);
    return len(p - (t.a + s * ab));
  }
  D3 cp = p - t.c;
  double d5 = dot(ab, cp), d6 = dot(ac, cp);
  if (d6 >= 0 && d5 <= d6) return len(p - t.c);
  double vb = d5 * d2 - d1 * d6;
  if (vb <= 0 && d2 >= 0 && d6 <= 0) {
    double s = d2 / (d2 - d6);
    return len(p - (t.a + s * ac));
  }
  double va = d3 * d6 - d5 * d4;
  if (va <= 0 && (d4 - d3) >= 0 && (d5 - d6) >= 0) {
    double s = (d4 - d3) / ((d4 - d3) + (d5 - d6));
    return len(p - (t.b + s * (t.c - t.b)));
  }
  double den = 1.0 / (va + vb + vc);
  double v = vb * den, w = vc * den;
  return len(p - (t.a + v * ab + w * ac));
}

// distance between segments p1q1 and p2q2 (clamped closest parameters)
double seg_seg_dist(D3 p1, D3 q1, D3 p2, D3 q2) {
  D3 d1 = q1 - p1, d2 = q2 - p2, r = p1 - p2;
  double a = dot(d1, d1), e = dot(d2, d2), f = dot(d2, r);
  double s, t;
  if (a <= 1e-30 && e <= 1e-30) return len(r);
  if (a <= 1e-30) {
    s = 0;
    t = clamp01(f / e);
  } else {
    double c = dot(d1, r);
    if (e <= 1e-30) {
      t = 0;
      s = clamp01(-c / a);
    } else {
      double b = dot(d1, d2);
      double den = a * e - b * b;
      s = den > 1e-30 * a * e ? clamp01((b * f - c * e) / den) : 0.0;
      t = (b * s + f) / e;
      if (t < 0) {
        t = 0;
        s = clamp01(-c / a);
      } else if (t > 1) {
        t = 1;
        s = clamp01((b - c) / a);
      }
    }
  }
  return len((p1 + s * d1) - (p2 + t * d2));
}

double tri_tri_dist(const Tri3& A, const Tri3& B) {
  const D3 av[3] = {A.a, A.b, A.c}, bv[3] = {B.a, B.b, B.c};
  for (int i = 0; i < 3; ++i) {
    if (segment_hits(av[i], av[(i + 1) % 3], B)) return 0.0;
    if (segment_hits(bv[i], bv[(i + 1) % 3], A)) return 0.0;
  }
  double d = INFINITY;
  for (int i = 0; i < 3; ++i) {
    d = std::min(d, point_tri_dist(av[i], B));
    d = std::min(d, point_tri_dist(bv[i], A));
    for (int j = 0; j < 3; ++j)
      d = std::min(d, seg_seg_dist(av[i], av[(i + 1) % 3], bv[j], bv[(j + 1) % 3]));
  }
  return d;
}

// parity probe directions (unit vectors, generic)
const double kProbe[8][3] = {
    {0.3420201433256687, 0.4698463103929542, 0.8137976813493738},
    {-0.6123724356957945, 0.6123724356957945, 0.5000000000000001},
    {0.5265407233266235, -0.2807702340418462, -0.8024434918893496},
    {-0.2588190451025208, -0.9153482049516813, 0.3085601688130047},
    {0.8717797887081347, 0.1889822365046136, -0.4520064213127209},
    {-0.7745966692414834, -0.3162277660168379, -0.5477225575051661},
    {0.1543033499620919, 0.7715167498104596, -0.6172133998483676},
    {0.6928203230275509, -0.6, 0.4},
};

enum { kMiss = 0, kHit = 1, kDegenerate = 2 };

// ray o + t d, t > 0, against a facet; edge/vertex/in-plane grazing => degenerate
int probe_facet(D3 o, D3 d, const Tri3& t, double ext, double& th) {
  D3 e1 = t.b - t.a, e2 = t.c - t.a;
  D3 n = cross(e1, e2);
  D3 p = cross(d, e2);
  double det = dot(e1, p);
  D3 s = o - t.a;
  if (fabs(det) <= 1e-13 * len(e1) * len(e2)) {
    return fabs(dot(s, n)) <= 1e-11 * len(n) * ext ? kDegenerate : kMiss;
  }
  double inv = 1.0 / det;
  double u = dot(s, p) * inv;
  D3 q = cross(s, e1);
  double v = dot(d, q) * inv;
  double w = 1.0 - u - v;
  const double tol = 1e-10;
  if (u < -tol || v < -tol || w < -tol) return kMiss;
  th = dot(e2, q) * inv;
  if (th < -1e-11 * ext) return kMiss;
  if (u < tol || v < tol || w < tol || th <= 1e-11 * ext) return kDegenerate;
  return kHit;
}

int fail(std::string& err, int code, const std::string& msg) {
  err = msg;
  return code;
}

}  // namespace

int prepare_mesh(const float* xyz, int64_t nv, const int32_t* tri, const int32_t* tri_region,
                 int64_t nt, int32_t n_regions, double min_gap, bool validate, int bvh_method,
                 double split_budget, PreparedMesh& out, std::string& err) {
  if (!xyz || !tri || !tri_region || nv < 3 || nt < 1)
    return fail(err, GADEP_E_ARG, "mesh: null array or empty mesh");
  if (n_regions < 2 || n_regions > kMaxRegions)
    return fail(err, GADEP_E_ARG, "mesh: n_regions must be in [2, 64]");
  if (nt > (int64_t(1) << 27)) return fail(err, GADEP_E_ARG, "mesh: too many facets");
  if (bvh_method != 0 && bvh_method != 1) return fail(err, GADEP_E_ARG, "mesh: bvh_method");

  // ---- basic checks
  std::vector<D3> v(static_cast<size_t>(nv));
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = 0; i < nv; ++i) {
    double x = xyz[3 * i], y = xyz[3 * i + 1], z = xyz[3 * i + 2];
    if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z))
      return fail(err, GADEP_E_MESH_DEGENERATE, "mesh: non-finite vertex " + std::to_string(i));
    v[i] = {x, y, z};
    lo[0] = std::min(lo[0], x), lo[1] = std::min(lo[1], y), lo[2] = std::min(lo[2], z);
    hi[0] = std::max(hi[0], x), hi[1] = std::max(hi[1], y), hi[2] = std::max(hi[2], z);
  }
  const double ext = sqrt((hi[0] - lo[0]) * (hi[0] - lo[0]) + (hi[1] - lo[1]) * (hi[1] - lo[1]) +
                          (hi[2] - lo[2]) * (hi[2] - lo[2]));
  std::vector<int32_t> tv(tri, tri + 3 * nt);
  for (int64_t f = 0; f < nt; ++f) {
    for (int k = 0; k < 3; ++k)
      if (tv[3 * f + k] < 0 || tv[3 * f + k] >= nv)
        return fail(err, GADEP_E_ARG, "mesh: vertex index out of range in facet " + std::to_string(f));
    if (tri_region[f] < 1 || tri_region[f] >= n_regions)
      return fail(err, GADEP_E_ARG, "mesh: facet region out of range in facet " + std::to_string(f));
    D3 a = v[tv[3 * f]], b = v[tv[3 * f + 1]], c = v[tv[3 * f + 2]];
    if (len(cross(b - a, c - a)) <= 0.0)
      return fail(err, GADEP_E_MESH_DEGENERATE, "mesh: zero-area facet " + std::to_string(f));
  }

  // ---- edges: each directed edge once, its reverse once, same region
  std::vector<int32_t> parent(static_cast<size_t>(nt));
  std::iota(parent.begin(), parent.end(), 0);
  auto find = [&](int32_t x) {
    while (parent[x] != x) x = parent[x] = parent[parent[x]];
    return x;
  };
  {
    std::unordered_map<uint64_t, int32_t> edge;
    edge.reserve(static_cast<size_t>(3 * nt));
    for (int64_t f = 0; f < nt; ++f)
      for (int k = 0; k < 3; ++k) {
        uint32_t a = tv[3 * f + k], b = tv[3 * f + (k + 1) % 3];
        uint64_t key = (uint64_t(a) << 32) | b;
        if (!edge.emplace(key, static_cast<int32_t>(f)).second) {
          if (validate)
            return fail(err, GADEP_E_MESH_ORIENT,
                        "mesh: directed edge used twice (inconsistent winding) at facet " +
                            std::to_string(f));
        }
      }
    for (int64_t f = 0; f < nt; ++f)
      for (int k = 0; k < 3; ++k) {
        uint32_t a = tv[3 * f + k], b = tv[3 * f + (k + 1) % 3];
        auto it = edge.find((uint64_t(b) << 32) | a);
        if (it == edge.end()) {
          if (validate)
            return fail(err, GADEP_E_MESH_OPEN,
                        "mesh: open edge at facet " + std::to_string(f) + " (region " +
                            std::to_string(tri_region[f]) + ")");
          continue;
        }
        if (tri_region[it->second] != tri_region[f] && validate)
          return fail(err, GADEP_E_MESH_OVERLAP,
                      "mesh: facets of regions " + std::to_string(tri_region[f]) + " and " +
                          std::to_string(tri_region[it->second]) + " share an edge");
        int32_t ra = find(static_cast<int32_t>(f)), rb = find(it->second);
        if (ra != rb) parent[ra] = rb;
      }
  }

  // ---- shells
  std::vector<int32_t> shell(static_cast<size_t>(nt), -1);
  std::vector<int32_t> shell_first;  // first facet of each shell
  {
    std::unordered_map<int32_t, int32_t> id;
    for (int64_t f = 0; f < nt; ++f) {
      int32_t r = find(static_cast<int32_t>(f));
      auto it = id.find(r);
      if (it == id.end()) {
        it = id.emplace(r, static_cast<int32_t>(shell_first.size())).first;
        shell_first.push_back(static_cast<int32_t>(f));
      }
      shell[f] = it->second;
    }
  }
  const int32_t ns = static_cast<int32_t>(shell_first.size());
  std::vector<double> vol(ns, 0.0);
  std::vector<int64_t> nf(ns, 0);
  for (int64_t f = 0; f < nt; ++f) {
    D3 a = v[tv[3 * f]], b = v[tv[3 * f + 1]], c = v[tv[3 * f + 2]];
    vol[shell[f]] += dot(a, cross(b, c)) / 6.0;
    nf[shell[f]]++;
  }
  int32_t genus_max = 0;
  {
    // Euler characteristic per shell: V - E + F, E = 3F/2 for a closed shell
    std::vector<std::vector<int32_t>> sv(ns);
    for (int64_t f = 0; f < nt; ++f)
      for (int k = 0; k < 3; ++k) sv[shell[f]].push_back(tv[3 * f + k]);
    for (int32_t s = 0; s < ns; ++s) {
      auto& x = sv[s];
      std::sort(x.begin(), x.end());
      int64_t nvs = std::unique(x.begin(), x.end()) - x.begin();
      int64_t chi = nvs - 3 * nf[s] / 2 + nf[s];
      genus_max = std::max<int32_t>(genus_max, static_cast<int32_t>((2 - chi) / 2));
    }
  }
  if (validate)
    for (int32_t s = 0; s < ns; ++s)
      if (!(vol[s] > 0))
        return fail(err, GADEP_E_MESH_ORIENT,
                    "mesh: shell of region " + std::to_string(tri_region[shell_first[s]]) +
                        " has non-positive signed volume (wound inward)");

  // ---- BVH
  std::vector<Ref> refs(static_cast<size_t>(nt));
  for (int64_t f = 0; f < nt; ++f) {
    Ref& r = refs[f];
    r.box.reset();
    for (int k = 0; k < 3; ++k) r.box.grow(xyz + 3 * tv[3 * f + k]);
    for (int a = 0; a < 3; ++a) r.c[a] = 0.5f * (r.box.lo[a] + r.box.hi[a]);
    r.id = static_cast<int32_t>(f);
  }
  const std::vector<Ref> refs_of = refs;  // whole-facet references by facet
  Builder builder(refs, bvh_method);
  builder.run(out.nodes, out.depth, out.sah);
  out.order.resize(static_cast<size_t>(nt));
  for (int64_t i = 0; i < nt; ++i) out.order[i] = refs[i].id;

  auto facet = [&](int32_t f) {
    return Tri3{v[tv[3 * f]], v[tv[3 * f + 1]], v[tv[3 * f + 2]]};
  };
  HostQuery q(out.nodes, out.order, 1e-9 * ext + 1e-12);

  // ---- shells must not intersect or come closer than min_gap
  double gap_seen = INFINITY;
  // candidate pairs: facets of different shells whose boxes lie within `reach`;
  // the smallest distance among them is reported (exact when below reach)
  const double reach = std::max(4.0 * min_gap, 1e-3);
  if (validate && ns > 1) {
    // facets in contiguous ranges, one per worker thread; the first offending
    // facet in index order is the one reported
    const int nth = worker_count(nt);
    std::vector<double> gap(nth, INFINITY);
    std::vector<int64_t> bad_f(nth, -1);
    std::vector<int32_t> bad_g(nth, -1);
    auto work = [&](int w) {
    for (int64_t f = nt * w / nth, fe = nt * (w + 1) / nth; f < fe; ++f) {
      Tri3 A = facet(static_cast<int32_t>(f));
      double blo[3], bhi[3];
      const D3 p[3] = {A.a, A.b, A.c};
      for (int a = 0; a < 3; ++a) {
        double mn = INFINITY, mx = -INFINITY;
        for (int k = 0; k < 3; ++k) {
          double c = a == 0 ? p[k].x : (a == 1 ? p[k].y : p[k].z);
          mn = std::min(mn, c);
          mx = std::max(mx, c);
        }
        blo[a] = mn - reach;
        bhi[a] = mx + reach;
      }
      int bad = -1;
      q.box_all(blo, bhi, [&](int32_t g) {
        if (bad >= 0 || g <= f || shell[g] == shell[f]) return;
        double d = tri_tri_dist(A, facet(g));
        gap[w] = std::min(gap[w], d);
        if (d < min_gap) bad = g;
      });
      if (bad >= 0) {
        bad_f[w] = f;
        bad_g[w] = bad;
        return;
      }
    }
    };
    run_workers(nth, work);
    for (int w = 0; w < nth; ++w) gap_seen = std::min(gap_seen, gap[w]);
    for (int w = 0; w < nth; ++w)
      if (bad_f[w] >= 0) {
        const int64_t f = bad_f[w];
        const int32_t bad = bad_g[w];
        return fail(err, GADEP_E_MESH_OVERLAP,
                    "mesh: shells of regions " + std::to_string(tri_region[f]) + " and " +
                        std::to_string(tri_region[bad]) + " intersect or are closer than the "
                        "minimum gap (facets " + std::to_string(f) + ", " + std::to_string(bad) + ")");
      }
  }

  // ---- topology: region outside each shell by the parity rule
  std::vector<int32_t> container(ns, 0);
  for (int32_t s = 0; s < ns; ++s) {
    Tri3 t0 = facet(shell_first[s]);
    D3 o = (1.0 / 3.0) * (t0.a + t0.b + t0.c);
    bool done = false;
    for (int k = 0; k < 8 && !done; ++k) {
      D3 d{kProbe[k][0], kProbe[k][1], kProbe[k][2]};
      d = (1.0 / len(d)) * d;
      uint64_t parity = 0;
      double first[kMaxRegions];
      for (double& x : first) x = INFINITY;
      bool degenerate = false;
      q.ray_all(o, d, [&](int32_t g) {
        if (degenerate || shell[g] == s) return;
        double th;
        int r = probe_facet(o, d, facet(g), ext, th);
        if (r == kDegenerate) degenerate = true;
        if (r != kHit) return;
        int32_t rg = tri_region[g];
        parity ^= uint64_t(1) << rg;
        first[rg] = std::min(first[rg], th);
      });
      if (degenerate) continue;
      int32_t best = 0;
      double tb = INFINITY;
      for (int32_t r = 1; r < n_regions; ++r)
        if (((parity >> r) & 1) && first[r] < tb) {
          tb = first[r];
          best = r;
        }
      container[s] = best;
      done = true;
    }
    if (!done) return fail(err, GADEP_E_TOPOLOGY, "mesh: every parity probe was degenerate");
    const int32_t own = tri_region[shell_first[s]];
    if (validate && container[s] == own)
      return fail(err, GADEP_E_TOPOLOGY,
                  "mesh: a shell of region " + std::to_string(own) +
                      " lies inside another shell of the same region");
  }

  // ---- is the world bounded by one convex shell?
  int32_t top = -1;
  {
    int32_t n_top = 0;
    for (int32_t s = 0; s < ns; ++s)
      if (container[s] == 0) {
        top = s;
        ++n_top;
      }
    out.convex_exit = false;
    if (n_top == 1) {
      std::vector<int32_t> fs, vs;
      for (int64_t f = 0; f < nt; ++f)
        if (shell[f] == top) {
          fs.push_back(static_cast<int32_t>(f));
          for (int k = 0; k < 3; ++k) vs.push_back(tv[3 * f + k]);
        }
      std::sort(vs.begin(), vs.end());
      vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
      if (static_cast<double>(fs.size()) * static_cast<double>(vs.size()) <= 2e8) {
        bool convex = true;
        for (size_t i = 0; i < fs.size() && convex; ++i) {
          Tri3 t = facet(fs[i]);
          D3 n = cross(t.b - t.a, t.c - t.a);
          const double tol = 1e-9 * len(n) * ext;
          for (int32_t vi : vs)
            if (dot(v[vi] - t.a, n) > tol) {
              convex = false;
              break;
            }
        }
        out.convex_exit = convex;
      }
    }
  }

  // ---- exit planes of that shell
  out.planes.clear();
  if (out.convex_exit) {
    std::vector<D3> pn;
    std::vector<double> pd;
    bool few = true;
    for (int64_t f = 0; f < nt && few; ++f) {
      if (shell[f] != top) continue;
      Tri3 t = facet(static_cast<int32_t>(f));
      D3 n = cross(t.b - t.a, t.c - t.a);
      n = (1.0 / len(n)) * n;
      const double d = dot(n, (1.0 / 3.0) * (t.a + t.b + t.c));
      bool seen = false;
      for (size_t k = 0; k < pn.size() && !seen; ++k)
        seen = dot(n, pn[k]) > 1.0 - 1e-12 && fabs(d - pd[k]) <= 1e-9 * ext;
      if (seen) continue;
      if (static_cast<int>(pn.size()) == kMaxExitPlanes) {
        few = false;
        break;
      }
      pn.push_back(n);
      pd.push_back(d);
    }
    if (few) {
      out.outer_region = tri_region[shell_first[top]];
      for (int a = 0; a < 3; ++a) {
        out.outer_lo[a] = INFINITY;
        out.outer_hi[a] = -INFINITY;
      }
      for (int64_t f = 0; f < nt; ++f) {
        if (shell[f] != top) continue;
        for (int k = 0; k < 3; ++k) {
          const float* p = xyz + 3 * tv[3 * f + k];
          for (int a = 0; a < 3; ++a) {
            out.outer_lo[a] = std::min(out.outer_lo[a], p[a]);
            out.outer_hi[a] = std::max(out.outer_hi[a], p[a]);
          }
        }
      }
      for (size_t k = 0; k < pn.size(); ++k) {
        out.planes.push_back(static_cast<float>(pn[k].x));
        out.planes.push_back(static_cast<float>(pn[k].y));
        out.planes.push_back(static_cast<float>(pn[k].z));
        out.planes.push_back(static_cast<float>(pd[k]));
      }
    }
  }

  // ---- transport BVHs (spatial splits), one per region over the facets
  // that bound it, plus the outer region's without the outermost shell
  {
    std::vector<int32_t> own(static_cast<size_t>(nt)), outside_of(static_cast<size_t>(nt));
    for (int64_t f = 0; f < nt; ++f) {
      own[f] = tri_region[f];
      outside_of[f] = container[shell[f]];
    }
    const bool with_planes = !out.planes.empty();
    const int32_t n_bvh = n_regions + (with_planes ? 1 : 0);
    std::vector<std::vector<Ref>> sets(static_cast<size_t>(n_bvh));
    for (int64_t f = 0; f < nt; ++f) {
      sets[own[f]].push_back(refs_of[f]);
      if (outside_of[f] != own[f]) sets[outside_of[f]].push_back(refs_of[f]);
      if (with_planes && shell[f] != top &&
          (own[f] == out.outer_region || outside_of[f] == out.outer_region))
        sets[n_regions].push_back(refs_of[f]);
    }
    struct Built {
      std::vector<BvhNode> nodes;
      std::vector<int32_t> ids;
      int32_t depth = 0;
      double sah = 0.0;
    };
    std::vector<Built> built(static_cast<size_t>(n_bvh));
    // largest sets first, one at a time per worker thread
    std::vector<int32_t> todo;
    for (int32_t b = 0; b < n_bvh; ++b)
      if (!sets[b].empty()) todo.push_back(b);
    std::sort(todo.begin(), todo.end(), [&](int32_t x, int32_t y) {
      return sets[x].size() > sets[y].size() || (sets[x].size() == sets[y].size() && x < y);
    });
    std::atomic<size_t> next{0};
    auto work = [&](int) {
      for (size_t k = next++; k < todo.size(); k = next++) {
        const int32_t b = todo[k];
        const int64_t n = static_cast<int64_t>(sets[b].size());
        const int64_t budget = static_cast<int64_t>(split_budget * static_cast<double>(n));
        SplitBuilder sb(xyz, tv.data(), n + budget, nt >= SplitBuilder::kPieceMinFacets);
        Built& o = built[b];
        sb.run(std::move(sets[b]), o.nodes, o.ids, o.depth, o.sah);
      }
    };
    run_workers(std::min<int>(worker_count(nt), static_cast<int>(todo.size())), work);
    out.trans_nodes.clear();
    out.trans_tris.clear();
    out.trans_root.assign(static_cast<size_t>(n_bvh), -1);
    out.trans_depth = 0;
    out.trans_sah = 0.0;
    for (int32_t b = 0; b < n_bvh; ++b) {
      const Built& o = built[b];
      if (o.nodes.empty()) continue;
      const int32_t node_off = static_cast<int32_t>(out.trans_nodes.size());
      const int64_t slot_off = static_cast<int64_t>(out.trans_tris.size());
      out.trans_root[b] = node_off;
      for (BvhNode nd : o.nodes) {
        for (int c = 0; c < 2; ++c) {
          if (nd.child[c] >= 0) {
            nd.child[c] += node_off;
          } else {
            const int32_t x = ~nd.child[c];
            nd.child[c] = leaf_code((x >> 3) + slot_off, x & 7);
          }
        }
        out.trans_nodes.push_back(nd);
      }
      for (int32_t id : o.ids) {
        TriRec r{};
        r.orig = id;
        out.trans_tris.push_back(r);
      }
      out.trans_depth = std::max(out.trans_depth, o.depth);
      out.trans_sah += o.sah;
    }
    for (int a = 0; a < 3; ++a) {
      out.trans_lo[a] = INFINITY;
      out.trans_hi[a] = -INFINITY;
    }
    if (with_planes && out.trans_root[n_regions] >= 0) {
      const BvhNode& root = out.trans_nodes[out.trans_root[n_regions]];
      for (int a = 0; a < 3; ++a) {
        out.trans_lo[a] = std::min(root.lmin[a], root.rmin[a]);
        out.trans_hi[a] = std::max(root.lmax[a], root.rmax[a]);
      }
    }
  }

  // ---- outputs
  out.outside.resize(static_cast<size_t>(nt));
  out.shell = shell;
  for (int64_t f = 0; f < nt; ++f) out.outside[f] = container[shell[f]];
  out.tris.resize(static_cast<size_t>(nt));
  auto record = [&](int32_t f, TriRec& r) {
    for (int k = 0; k < 3; ++k) {
      const float* p = xyz + 3 * tv[3 * f + k];
      float* dst = k == 0 ? r.v0 : (k == 1 ? r.v1 : r.v2);
      dst[0] = p[0], dst[1] = p[1], dst[2] = p[2];
    }
    r.regions = uint32_t(tri_region[f]) | (uint32_t(out.outside[f]) << 16);
    r.orig = f;
    r.pad = 0;
  };
  for (int64_t i = 0; i < nt; ++i) record(out.order[i], out.tris[i]);
  for (TriRec& r : out.trans_tris) record(r.orig, r);
  out.n_shells = ns;
  out.genus_max = genus_max;
  out.min_gap = gap_seen;
  return GADEP_OK;
}

}  // namespace gadep

// ---------------------------------------------------------------------------
// host-only export of the preparation (no device, no context)

using namespace gadep;

extern "C" gadep_status gadep_mesh_prepare(const float* xyz, int64_t nv, const int32_t* tri,
                                           const int32_t* tri_region, int64_t nt,
                                           int32_t n_regions, double min_gap_mm, int32_t validate,
                                           int32_t bvh_method, double split_budget,
                                           int32_t* tri_outside, int32_t* tri_shell,
                                           void* nodes_out, int64_t cap_nodes, int32_t* tri_order,
                                           int64_t cap_slots, gadep_mesh_info* info, char* err,
                                           int32_t err_len) {
  if (bvh_method < 0 || bvh_method > 2 || !(split_budget >= 0) || split_budget > 16) {
    if (err && err_len > 0) {
      strncpy(err, "mesh: bvh_method or split_budget out of range", static_cast<size_t>(err_len) - 1);
      err[err_len - 1] = 0;
    }
    return GADEP_E_ARG;
  }
  PreparedMesh pm;
  std::string e;
  int rc = prepare_mesh(xyz, nv, tri, tri_region, nt, n_regions, min_gap_mm, validate != 0,
                        bvh_method == 1 ? 1 : 0, split_budget, pm, e);
  if (err && err_len > 0) {
    strncpy(err, e.c_str(), static_cast<size_t>(err_len) - 1);
    err[err_len - 1] = 0;
  }
  if (rc != GADEP_OK) return static_cast<gadep_status>(rc);
  const bool trans = bvh_method == 2;
  const std::vector<BvhNode>& nodes = trans ? pm.trans_nodes : pm.nodes;
  const int64_t n_slots = trans ? static_cast<int64_t>(pm.trans_tris.size()) : nt;
  if (info) {
    info->n_shells = pm.n_shells;
    info->genus_max = pm.genus_max;
    info->n_nodes = static_cast<int64_t>(nodes.size());
    info->depth = trans ? pm.trans_depth : pm.depth;
    info->sah_cost = trans ? pm.trans_sah : pm.sah;
    info->n_slots = n_slots;
    info->min_gap_mm = pm.min_gap;
    info->convex_exit = pm.convex_exit ? 1 : 0;
    info->n_exit_planes = static_cast<int32_t>(pm.planes.size() / 4);
    for (int32_t r = 0; r <= GADEP_MAX_REGIONS; ++r)
      info->region_root[r] = trans && r < static_cast<int32_t>(pm.trans_root.size()) ? pm.trans_root[r]
                                                                                     : -1;
  }
  if (tri_outside) memcpy(tri_outside, pm.outside.data(), pm.outside.size() * 4);
  if (tri_shell) memcpy(tri_shell, pm.shell.data(), pm.shell.size() * 4);
  if (tri_order) {
    if (cap_slots < n_slots) return GADEP_E_ARG;
    if (trans)
      for (int64_t i = 0; i < n_slots; ++i) tri_order[i] = pm.trans_tris[i].orig;
    else
      memcpy(tri_order, pm.order.data(), pm.order.size() * 4);
  }
  if (nodes_out) {
    if (cap_nodes < static_cast<int64_t>(nodes.size())) return GADEP_E_ARG;
    memcpy(nodes_out, nodes.data(), nodes.size() * sizeof(BvhNode));
  }
  return GADEP_OK;
}

