// Host induction of one M5P model tree (Section 3.4, after Quinlan's M5):
//
//  grow     binary splits z_j <= t, t halfway between two adjacent distinct
//           training values; the split kept maximises the standard-deviation
//           reduction sd(T) - |T_l|/|T| sd(T_l) - |T_r|/|T| sd(T_r)
//           (population sd of the labels).  Every feature's case order is
//           sorted once; a split partitions each order stably, so a node's
//           cases stay one contiguous, sorted range of every order and a scan
//           over them needs no sort.  Nodes with fewer than 2 min_leaf cases or
//           with label sd at most sd_frac of the root's are leaves.
//  models   least squares with an intercept at every node, on the features
//           tested inside its subtree (a constant at a leaf), from centred
//           normal equations and a Cholesky factorisation taken in feature
//           order, which leaves out a feature whose pivot (its residual sum
//           of squares given the features kept before it) is at most 1e-9 of
//           its own sum of squares; estimated error mean |residual| *
//           (n + v) / (n - v), v the kept parameters.
//  prune    bottom-up: a node whose own model's estimate is no larger than
//           the case-weighted estimate of its pruned children becomes a leaf.
//  smooth   from a leaf up to the root, p <- (n_c p + K q) / (n_c + K) with q
//           the ancestor's model and n_c the cases of the child on the path;
//           folded into one linear model per leaf.
//
// Ties: split candidates within tie * sd(root) of the best SDR are equal and
// the first in (feature, threshold) order is kept; a pruning comparison
// within the same margin prunes.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <numeric>
#include <vector>

#include "m5p.hpp"

namespace sugg {
namespace {

struct GNode {
  int64_t lo = 0, hi = 0;   // the node's cases: positions [lo, hi) of every feature order
  int32_t feat = -1;
  double thr = 0.0;
  int32_t left = -1, right = -1;
};

struct NodeModel {
  std::vector<int32_t> A;   // features
  std::vector<double> w;    // coefficients on A (0 for a feature left out)
  double b = 0.0;           // intercept
  double est = 0.0;         // M5 error estimate
  int kept = 0;             // features with a coefficient
};

class Grower {
 public:
  Grower(const double* Z, int64_t ldz, const int32_t* rows, const double* y, int64_t n, int E, const M5pParams& p)
      : Z_(Z), ldz_(ldz), rows_(rows), y_(y), n_(n), E_(E), p_(p) {}

  M5pHostTree run() {
    presort();
    sd_root_ = label_sd(0, n_);
    tol_ = p_.tie * sd_root_;
    grow();
    models();
    prune();
    return emit();
  }

 private:
  const double* Z_;
  int64_t ldz_;
  const int32_t* rows_;
  const double* y_;
  int64_t n_;
  int E_;
  M5pParams p_;
  double sd_root_ = 0.0, tol_ = 0.0;
  std::vector<int32_t> ord_;      // [E][n] case ids by ascending feature value
  std::vector<double> val_;       // [E][n] the values in that order
  std::vector<GNode> nodes_;
  std::vector<NodeModel> model_;
  std::vector<char> is_leaf_;

  double z(int64_t i, int j) const { return Z_[(int64_t)rows_[i] * ldz_ + j]; }

  void presort() {
    ord_.resize((size_t)E_ * n_);
    val_.resize((size_t)E_ * n_);
    for (int j = 0; j < E_; ++j) {
      int32_t* o = ord_.data() + (size_t)j * n_;
      std::iota(o, o + n_, 0);
      std::stable_sort(o, o + n_, [&](int32_t a, int32_t b) { return z(a, j) < z(b, j); });
      double* v = val_.data() + (size_t)j * n_;
      for (int64_t p = 0; p < n_; ++p) v[p] = z(o[p], j);
    }
  }

  // population sd of the labels of positions [lo, hi) (any feature order)
  double label_sd(int64_t lo, int64_t hi) const {
    const int64_t m = hi - lo;
    if (m <= 0) return 0.0;
    const int32_t* o = ord_.data();
    double s = 0.0;
    for (int64_t p = lo; p < hi; ++p) s += y_[o[p]];
    const double mean = s / (double)m;
    double q = 0.0;
    for (int64_t p = lo; p < hi; ++p) {
      const double d = y_[o[p]] - mean;
      q += d * d;
    }
    return std::sqrt(q / (double)m);
  }

  // SDR of every admissible split of feature j over [lo, hi); calls f(pos, sdr)
  // with pos the last left position.
  template <typename F>
  void scan(int j, int64_t lo, int64_t hi, double mean, double sd_t, F&& f) const {
    const int32_t* o = ord_.data() + (size_t)j * n_;
    const double* v = val_.data() + (size_t)j * n_;
    const int64_t m = hi - lo;
    double t1 = 0.0, t2 = 0.0;
    for (int64_t p = lo; p < hi; ++p) {
      const double d = y_[o[p]] - mean;
      t1 += d;
      t2 += d * d;
    }
    double s1 = 0.0, s2 = 0.0;
    const int64_t last = hi - p_.min_leaf;   // the left side may end at positions up to last - 1
    for (int64_t p = lo; p < last; ++p) {
      const double d = y_[o[p]] - mean;
      s1 += d;
      s2 += d * d;
      const int64_t nl = p - lo + 1;
      if (nl < p_.min_leaf || !(v[p] < v[p + 1])) continue;
      const double fl = (double)nl, fr = (double)(m - nl);
      const double r1 = t1 - s1, r2 = t2 - s2;
      const double sdl = std::sqrt(std::max(s2 / fl - (s1 / fl) * (s1 / fl), 0.0));
      const double sdr = std::sqrt(std::max(r2 / fr - (r1 / fr) * (r1 / fr), 0.0));
      f(p, sd_t - (fl / (double)m) * sdl - (fr / (double)m) * sdr);
    }
  }

  void grow() {
    struct Pending {
      int64_t lo, hi;
      int32_t parent;
      int side;
    };
    std::vector<Pending> stack{{0, n_, -1, 0}};
    std::vector<char> go_left(n_);
    std::vector<int32_t> tmp_o(n_);
    std::vector<double> tmp_v(n_);
    std::vector<double> fmax(E_);
    while (!stack.empty()) {
      const Pending pd = stack.back();
      stack.pop_back();
      const int32_t me = (int32_t)nodes_.size();
      GNode nd;
      nd.lo = pd.lo;
      nd.hi = pd.hi;
      nodes_.push_back(nd);
      if (pd.parent >= 0) (pd.side == 0 ? nodes_[pd.parent].left : nodes_[pd.parent].right) = me;
      const int64_t m = pd.hi - pd.lo;
      if (m < 2 * (int64_t)p_.min_leaf) continue;
      const double sd_t = label_sd(pd.lo, pd.hi);
      if (sd_t <= p_.sd_frac * sd_root_) continue;
      double s = 0.0;
      for (int64_t p = pd.lo; p < pd.hi; ++p) s += y_[ord_[p]];
      const double mean = s / (double)m;
      const double ninf = -std::numeric_limits<double>::infinity();
      double best = ninf;
      for (int j = 0; j < E_; ++j) {
        double fm = ninf;
        scan(j, pd.lo, pd.hi, mean, sd_t, [&](int64_t, double r) { fm = std::max(fm, r); });
        fmax[j] = fm;
        best = std::max(best, fm);
      }
      if (!(best > ninf)) continue;
      int bj = -1;
      int64_t bp = -1;
      for (int j = 0; j < E_ && bj < 0; ++j) {
        if (!(fmax[j] >= best - tol_)) continue;
        scan(j, pd.lo, pd.hi, mean, sd_t, [&](int64_t p, double r) {
          if (bp < 0 && r >= best - tol_) bp = p;
        });
        if (bp >= 0) bj = j;
      }
      const double* v = val_.data() + (size_t)bj * n_;
      const double thr = 0.5 * (v[bp] + v[bp + 1]);
      nodes_[me].feat = bj;
      nodes_[me].thr = thr;
      // stable partition of every feature order of the range
      int64_t nl = 0;
      for (int64_t p = pd.lo; p < pd.hi; ++p) {
        const int32_t i = ord_[(size_t)bj * n_ + p];
        go_left[i] = z(i, bj) <= thr;
        nl += go_left[i];
      }
      for (int f = 0; f < E_; ++f) {
        int32_t* o = ord_.data() + (size_t)f * n_;
        double* vv = val_.data() + (size_t)f * n_;
        int64_t a = pd.lo, b = 0;
        for (int64_t p = pd.lo; p < pd.hi; ++p) {
          if (go_left[o[p]]) {
            o[a] = o[p];
            vv[a] = vv[p];
            ++a;
          } else {
            tmp_o[b] = o[p];
            tmp_v[b] = vv[p];
            ++b;
          }
        }
        std::copy(tmp_o.begin(), tmp_o.begin() + b, o + a);
        std::copy(tmp_v.begin(), tmp_v.begin() + b, vv + a);
      }
      stack.push_back({pd.lo + nl, pd.hi, me, 1});
      stack.push_back({pd.lo, pd.lo + nl, me, 0});   // popped first: preorder
    }
  }

  // least squares on A with an intercept over the node's cases
  NodeModel fit(const GNode& nd, std::vector<int32_t> A) const {
    NodeModel md;
    md.A = std::move(A);
    const int a = (int)md.A.size();
    const int64_t m = nd.hi - nd.lo;
    const int32_t* cases = ord_.data() + nd.lo;
    std::vector<double> xm(a, 0.0);
    double ym = 0.0;
    for (int64_t p = 0; p < m; ++p) {
      const int32_t i = cases[p];
      ym += y_[i];
      for (int q = 0; q < a; ++q) xm[q] += z(i, md.A[q]);
    }
    ym /= (double)m;
    for (int q = 0; q < a; ++q) xm[q] /= (double)m;
    md.w.assign(a, 0.0);
    if (a > 0) {
      std::vector<double> G((size_t)a * a, 0.0), r(a, 0.0), x(a);
      for (int64_t p = 0; p < m; ++p) {
        const int32_t i = cases[p];
        for (int q = 0; q < a; ++q) x[q] = z(i, md.A[q]) - xm[q];
        const double yc = y_[i] - ym;
        for (int q = 0; q < a; ++q) {
          const double xq = x[q];
          double* g = G.data() + (size_t)q * a;
          for (int t = 0; t <= q; ++t) g[t] += xq * x[t];
          r[q] += xq * yc;
        }
      }
      md.kept = solve_dropping(G, r, a);
      md.w = r;
    }
    md.b = ym;
    for (int q = 0; q < a; ++q) md.b -= md.w[q] * xm[q];
    double sae = 0.0;
    for (int64_t p = 0; p < m; ++p) {
      const int32_t i = cases[p];
      double pr = md.b;
      for (int q = 0; q < a; ++q) pr += md.w[q] * z(i, md.A[q]);
      sae += std::fabs(y_[i] - pr);
    }
    const double v = (double)(md.kept + 1);
    md.est = (double)m > v ? ((double)m + v) / ((double)m - v) * (sae / (double)m)
                           : std::numeric_limits<double>::infinity();
    return md;
  }

  // G x = r for the centred Gram matrix G (lower triangle filled), by a
  // Cholesky factorisation in feature order that leaves out every feature
  // whose pivot is at most kDrop of its diagonal (x = 0 there).  Returns the
  // number of features kept.
  static int solve_dropping(std::vector<double>& G, std::vector<double>& r, int a) {
    constexpr double kDrop = 1e-9;
    std::vector<char> keep(a, 0);
    std::vector<double> diag(a);
    for (int q = 0; q < a; ++q) diag[q] = G[(size_t)q * a + q];
    int kept = 0;
    for (int q = 0; q < a; ++q) {
      for (int t = 0; t < q; ++t) {
        if (!keep[t]) continue;
        double s = G[(size_t)q * a + t];
        for (int u = 0; u < t; ++u)
          if (keep[u]) s -= G[(size_t)q * a + u] * G[(size_t)t * a + u];
        G[(size_t)q * a + t] = s / G[(size_t)t * a + t];
      }
      double s = diag[q];
      for (int u = 0; u < q; ++u)
        if (keep[u]) s -= G[(size_t)q * a + u] * G[(size_t)q * a + u];
      if (diag[q] > 0.0 && s > kDrop * diag[q]) {
        keep[q] = 1;
        G[(size_t)q * a + q] = std::sqrt(s);
        ++kept;
      }
    }
    for (int q = 0; q < a; ++q) {
      if (!keep[q]) continue;
      double s = r[q];
      for (int u = 0; u < q; ++u)
        if (keep[u]) s -= G[(size_t)q * a + u] * r[u];
      r[q] = s / G[(size_t)q * a + q];
    }
    for (int q = a - 1; q >= 0; --q) {
      if (!keep[q]) {
        r[q] = 0.0;
        continue;
      }
      double s = r[q];
      for (int u = q + 1; u < a; ++u)
        if (keep[u]) s -= G[(size_t)u * a + q] * r[u];
      r[q] = s / G[(size_t)q * a + q];
    }
    return kept;
  }

  void models() {
    const size_t nn = nodes_.size();
    const int words = (E_ + 63) / 64;
    std::vector<uint64_t> used(nn * words, 0);
    for (size_t k = nn; k-- > 0;) {   // children come after their parent
      const GNode& nd = nodes_[k];
      if (nd.feat < 0) continue;
      uint64_t* u = used.data() + k * words;
      const uint64_t* l = used.data() + (size_t)nd.left * words;
      const uint64_t* r = used.data() + (size_t)nd.right * words;
      for (int w = 0; w < words; ++w) u[w] = l[w] | r[w];
      u[nd.feat / 64] |= (uint64_t)1 << (nd.feat % 64);
    }
    model_.resize(nn);
    for (size_t k = 0; k < nn; ++k) {
      std::vector<int32_t> A;
      const uint64_t* u = used.data() + k * words;
      for (int j = 0; j < E_; ++j)
        if ((u[j / 64] >> (j % 64)) & 1) A.push_back(j);
      model_[k] = fit(nodes_[k], std::move(A));
    }
  }

  void prune() {
    const size_t nn = nodes_.size();
    is_leaf_.assign(nn, 0);
    std::vector<double> est(nn, 0.0);
    for (size_t k = nn; k-- > 0;) {
      const GNode& nd = nodes_[k];
      if (nd.feat < 0) {
        is_leaf_[k] = 1;
        est[k] = model_[k].est;
        continue;
      }
      const GNode& L = nodes_[nd.left];
      const GNode& R = nodes_[nd.right];
      const double sub = ((double)(L.hi - L.lo) * est[nd.left] + (double)(R.hi - R.lo) * est[nd.right]) /
                         (double)(nd.hi - nd.lo);
      if (model_[k].est <= sub + tol_) {
        is_leaf_[k] = 1;
        est[k] = model_[k].est;
      } else {
        est[k] = sub;
      }
    }
  }

  M5pHostTree emit() const {
    M5pHostTree t;
    const int W = E_ + 1;
    struct Visit {
      int32_t node, parent, side, depth;
    };
    std::vector<Visit> stack{{0, -1, 0, 0}};
    std::vector<int32_t> path;        // original node ids, root first
    std::vector<double> acc(W), q(W);
    while (!stack.empty()) {
      const Visit vs = stack.back();
      stack.pop_back();
      path.resize(vs.depth);
      path.push_back(vs.node);
      const GNode& nd = nodes_[vs.node];
      const int32_t me = (int32_t)t.feat.size();
      const bool leaf = is_leaf_[vs.node] != 0;
      t.feat.push_back(leaf ? -1 : nd.feat);
      t.thr.push_back(leaf ? 0.0 : nd.thr);
      t.left.push_back(-1);
      t.right.push_back(-1);
      t.leaf.push_back(-1);
      t.count.push_back(nd.hi - nd.lo);
      if (vs.parent >= 0) (vs.side == 0 ? t.left[vs.parent] : t.right[vs.parent]) = me;
      t.depth = std::max(t.depth, (int)vs.depth);
      if (!leaf) {
        stack.push_back({nd.right, me, 1, vs.depth + 1});
        stack.push_back({nd.left, me, 0, vs.depth + 1});
        continue;
      }
      // the smoothed model of this leaf: its own, blended towards the root
      expand(model_[vs.node], acc);
      for (int d = vs.depth - 1; d >= 0; --d) {
        const GNode& child = nodes_[path[d + 1]];
        const double nc = (double)(child.hi - child.lo);
        const double kk = p_.smooth_k;
        expand(model_[path[d]], q);
        for (int c = 0; c < W; ++c) acc[c] = (nc * acc[c] + kk * q[c]) / (nc + kk);
      }
      t.leaf[me] = t.leaves++;
      t.lw.insert(t.lw.end(), acc.begin(), acc.end());
    }
    return t;
  }

  void expand(const NodeModel& md, std::vector<double>& out) const {
    std::fill(out.begin(), out.end(), 0.0);
    for (size_t q = 0; q < md.A.size(); ++q) out[md.A[q]] = md.w[q];
    out[E_] = md.b;
  }
};

}  // namespace

M5pHostTree m5p_induce(const double* Z, int64_t ldz, const int32_t* rows, const double* y, int64_t n, int E,
                       const M5pParams& prm) {
  Grower g(Z, ldz, rows, y, n, E, prm);
  return g.run();
}

}  // namespace sugg
