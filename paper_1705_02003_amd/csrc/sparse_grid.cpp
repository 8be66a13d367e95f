// Host side of the method: the piecewise-linear hierarchical sparse-grid
// surrogate of iteration counts, surrogate-based grouping and classic
// surplus-driven refinement.
//
// Paper, Section 2.2 (hat functions, hierarchical surpluses, tensor-product
// basis, Smolyak level |l|, triangular surplus system, adaptivity) and
// Section 3.1 (order new samples by increasing predicted iterations and cut
// them into ensembles of S; the initial set keeps its generation order);
// Section 4, Test 1 footnote (pad the last ensemble by replicating its last
// sample).
//
// Floating-point evaluation order is fixed (this file is compiled with
// -ffp-contract=off): nodes are visited in canonical order (total level,
// level vector, index vector, each lexicographic); a term is c, multiplied by
// the 1-D hat values for dimensions 0..d-1, then added to the running sum.
// At grid nodes all quantities are dyadic and the results are exact.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <map>
#include <vector>

#include "ens.h"

namespace {

constexpr int kMaxLevel = 30;
constexpr int kMaxDim = 64;

struct Grid {
  int d = 0;
  int M = 0;
  std::vector<int32_t> lvl;   // [M][d]
  std::vector<int32_t> idx;   // [M][d]
  std::vector<int32_t> total; // [M]
  const int32_t* L(int m) const { return &lvl[(size_t)m * d]; }
  const int32_t* K(int m) const { return &idx[(size_t)m * d]; }
};

bool valid_1d(int32_t l, int32_t k) {
  if (l < 0 || l > kMaxLevel) return false;
  if (l == 0) return k == 0;
  if (l == 1) return k == 0 || k == 1;
  return k >= 0 && k < (int32_t(1) << (l - 1));
}

double coord_1d(int32_t l, int32_t k) {
  if (l == 0) return 0.0;
  if (l == 1) return k == 0 ? -1.0 : 1.0;
  return -1.0 + (double)(2 * k + 1) * std::ldexp(1.0, 1 - l);
}

double hat_1d(int32_t l, int32_t k, double y) {
  if (l == 0) return 1.0;
  const double yk = coord_1d(l, k);
  const double scale = (l == 1) ? 1.0 : std::ldexp(1.0, l - 1);
  const double v = 1.0 - scale * std::fabs(y - yk);
  return v > 0.0 ? v : 0.0;
}

// canonical order: total level, then level vector, then index vector
bool canon_less(const Grid& g, int a, int b) {
  if (g.total[a] != g.total[b]) return g.total[a] < g.total[b];
  const int32_t *la = g.L(a), *lb = g.L(b);
  for (int n = 0; n < g.d; ++n)
    if (la[n] != lb[n]) return la[n] < lb[n];
  const int32_t *ka = g.K(a), *kb = g.K(b);
  for (int n = 0; n < g.d; ++n)
    if (ka[n] != kb[n]) return ka[n] < kb[n];
  return false;
}

int load_grid(int32_t d, int32_t M, const int32_t* level, const int32_t* index, Grid& g) {
  if (d < 1 || d > kMaxDim || M < 0) return ENS_EINVAL;
  if (M > 0 && (!level || !index)) return ENS_EINVAL;
  g.d = d;
  g.M = M;
  g.lvl.assign(level, level + (size_t)M * d);
  g.idx.assign(index, index + (size_t)M * d);
  g.total.resize(M);
  for (int m = 0; m < M; ++m) {
    int t = 0;
    for (int n = 0; n < d; ++n) {
      if (!valid_1d(g.L(m)[n], g.K(m)[n])) return ENS_EINVAL;
      t += g.L(m)[n];
    }
    g.total[m] = t;
  }
  // reject duplicate nodes
  std::vector<int> order(M);
  for (int m = 0; m < M; ++m) order[m] = m;
  std::sort(order.begin(), order.end(), [&](int a, int b) { return canon_less(g, a, b); });
  for (int m = 1; m < M; ++m)
    if (!canon_less(g, order[m - 1], order[m])) return ENS_EINVAL;
  return ENS_OK;
}

std::vector<int> canonical_order(const Grid& g) {
  std::vector<int> order(g.M);
  for (int m = 0; m < g.M; ++m) order[m] = m;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return canon_less(g, a, b); });
  return order;
}

// sum over `nodes` (already in canonical order) of c_j psi_j(y)
double accumulate(const Grid& g, const std::vector<int>& nodes, const std::vector<double>& c,
                  const double* y) {
  double acc = 0.0;
  for (int j : nodes) {
    double t = c[j];
    const int32_t *l = g.L(j), *k = g.K(j);
    for (int n = 0; n < g.d; ++n) t = t * hat_1d(l[n], k[n], y[n]);
    acc = acc + t;
  }
  return acc;
}

void node_coords(const Grid& g, int m, double* y) {
  for (int n = 0; n < g.d; ++n) y[n] = coord_1d(g.L(m)[n], g.K(m)[n]);
}

// surpluses in input order; solved level by level (triangular system)
void surpluses(const Grid& g, const double* value, std::vector<double>& c) {
  c.assign(g.M, 0.0);
  const std::vector<int> order = canonical_order(g);
  std::vector<int> done;
  done.reserve(g.M);
  std::vector<double> y(g.d);
  size_t a = 0;
  while (a < order.size()) {
    size_t b = a;
    while (b < order.size() && g.total[order[b]] == g.total[order[a]]) ++b;
    for (size_t p = a; p < b; ++p) {
      const int m = order[p];
      node_coords(g, m, y.data());
      c[m] = value[m] - accumulate(g, done, c, y.data());
    }
    for (size_t p = a; p < b; ++p) done.push_back(order[p]);
    a = b;
  }
}

// Integral of a 1-D hierarchical basis function against the uniform density
// 1/2 on [-1, 1]: 1 at level 0 (the constant), 1/4 at level 1 (half a hat of
// unit base at the end points), 2^-l at level l >= 2 (a whole hat of
// half-width 2^(1-l)).
double weight_1d(int32_t l) {
  if (l == 0) return 1.0;
  if (l == 1) return 0.25;
  return std::ldexp(1.0, -l);
}

bool finite_all(const double* v, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(v[i])) return false;
  return true;
}

}  // namespace

extern "C" {

int ens_sg_coords(int32_t d, int32_t M, const int32_t* node_level, const int32_t* node_index,
                  double* y_out) {
  Grid g;
  int rc = load_grid(d, M, node_level, node_index, g);
  if (rc) return rc;
  if (M > 0 && !y_out) return ENS_EINVAL;
  for (int m = 0; m < M; ++m) node_coords(g, m, y_out + (size_t)m * d);
  return ENS_OK;
}

int ens_sg_surpluses(int32_t d, int32_t M, const int32_t* node_level, const int32_t* node_index,
                     const double* node_value, double* surplus_out) {
  Grid g;
  int rc = load_grid(d, M, node_level, node_index, g);
  if (rc) return rc;
  if (M > 0 && (!node_value || !surplus_out)) return ENS_EINVAL;
  if (!finite_all(node_value, (size_t)M)) return ENS_EINVAL;
  std::vector<double> c;
  surpluses(g, node_value, c);
  std::copy(c.begin(), c.end(), surplus_out);
  return ENS_OK;
}

int ens_sg_expectation(int32_t d, int32_t M, const int32_t* node_level, const int32_t* node_index,
                       const double* node_value, double* mean_out) {
  Grid g;
  int rc = load_grid(d, M, node_level, node_index, g);
  if (rc) return rc;
  if (M == 0 || !node_value || !mean_out) return ENS_EINVAL;
  if (!finite_all(node_value, (size_t)M)) return ENS_EINVAL;
  std::vector<double> c;
  surpluses(g, node_value, c);
  // the interpolant integrates term by term: sum_m c_m prod_n w(l_mn)
  double acc = 0.0;
  for (int m : canonical_order(g)) {
    double t = c[m];
    for (int n = 0; n < d; ++n) t = t * weight_1d(g.L(m)[n]);
    acc = acc + t;
  }
  *mean_out = acc;
  return ENS_OK;
}

int ens_group_samples(int32_t d, int32_t M, const int32_t* node_level, const int32_t* node_index,
                      const double* node_value, int32_t M_new, const double* y_new, int32_t S,
                      int32_t* groups_out, double* pred_out) {
  if (S < 1 || M_new < 0 || d < 1 || d > kMaxDim || M < 0) return ENS_EINVAL;
  if (M_new > 0 && (!y_new || !groups_out || !pred_out)) return ENS_EINVAL;
  Grid g;
  int rc = load_grid(d, M, node_level, node_index, g);
  if (rc) return rc;
  if (M > 0 && !node_value) return ENS_EINVAL;
  if (!finite_all(node_value, (size_t)M) || !finite_all(y_new, (size_t)M_new * d))
    return ENS_EINVAL;
  for (size_t i = 0; i < (size_t)M_new * d; ++i)
    if (y_new[i] < -1.0 || y_new[i] > 1.0) return ENS_EINVAL;
  if (M_new == 0) return ENS_OK;

  std::vector<int> order(M_new);
  for (int i = 0; i < M_new; ++i) order[i] = i;
  if (M == 0) {
    std::fill(pred_out, pred_out + M_new, 0.0);
  } else {
    std::vector<double> c;
    surpluses(g, node_value, c);
    const std::vector<int> canon = canonical_order(g);
    for (int i = 0; i < M_new; ++i) pred_out[i] = accumulate(g, canon, c, y_new + (size_t)i * d);
    std::sort(order.begin(), order.end(), [&](int a, int b) {
      if (pred_out[a] != pred_out[b]) return pred_out[a] < pred_out[b];
      return a < b;
    });
  }
  const int n_groups = (M_new + S - 1) / S;
  for (int gi = 0; gi < n_groups; ++gi) {
    const int base = gi * S;
    const int last = std::min(base + S, M_new) - 1;
    for (int s = 0; s < S; ++s) {
      const int pos = std::min(base + s, last);
      groups_out[(size_t)gi * S + s] = order[pos];
    }
  }
  return ENS_OK;
}

int ens_sg_refine(int32_t d, int32_t M, const int32_t* node_level, const int32_t* node_index,
                  const double* node_value, int32_t newest_level, double tau_rel, int32_t budget,
                  int32_t max_new, int32_t* new_level_out, int32_t* new_index_out,
                  int32_t* n_new_out) {
  if (!n_new_out || max_new < 0 || !std::isfinite(tau_rel) || tau_rel < 0.0) return ENS_EINVAL;
  Grid g;
  int rc = load_grid(d, M, node_level, node_index, g);
  if (rc) return rc;
  if (M == 0 || !node_value) return ENS_EINVAL;
  if (!finite_all(node_value, (size_t)M)) return ENS_EINVAL;
  *n_new_out = 0;

  std::vector<double> c;
  surpluses(g, node_value, c);
  double centre = 0.0;
  for (int m = 0; m < M; ++m)
    if (g.total[m] == 0) centre = node_value[m];
  const double tau = tau_rel * std::fabs(centre);

  // candidate children keyed by (level vector, index vector)
  typedef std::vector<int32_t> Key;  // [2d]: levels then indices
  std::map<Key, int> existing;
  for (int m = 0; m < M; ++m) {
    Key k(2 * d);
    std::copy(g.L(m), g.L(m) + d, k.begin());
    std::copy(g.K(m), g.K(m) + d, k.begin() + d);
    existing[k] = m;
  }
  std::map<Key, double> prio;
  for (int m = 0; m < M; ++m) {
    if (g.total[m] != newest_level || std::fabs(c[m]) < tau) continue;
    for (int n = 0; n < d; ++n) {
      const int32_t l = g.L(m)[n], k = g.K(m)[n];
      int32_t kids[2][2];
      int nk = 0;
      if (l == 0) {
        kids[0][0] = 1; kids[0][1] = 0; kids[1][0] = 1; kids[1][1] = 1; nk = 2;
      } else if (l == 1) {
        kids[0][0] = 2; kids[0][1] = k; nk = 1;
      } else {
        if (l + 1 > kMaxLevel) continue;
        kids[0][0] = l + 1; kids[0][1] = 2 * k; kids[1][0] = l + 1; kids[1][1] = 2 * k + 1; nk = 2;
      }
      for (int q = 0; q < nk; ++q) {
        Key key(2 * d);
        std::copy(g.L(m), g.L(m) + d, key.begin());
        std::copy(g.K(m), g.K(m) + d, key.begin() + d);
        key[n] = kids[q][0];
        key[d + n] = kids[q][1];
        if (existing.count(key)) continue;
        auto it = prio.find(key);
        const double p = std::fabs(c[m]);
        if (it == prio.end()) prio[key] = p;
        else if (p > it->second) it->second = p;
      }
    }
  }
  const int room = budget - M;
  if (room <= 0 || prio.empty()) return ENS_OK;

  // candidates as a grid for canonical comparisons
  Grid cg;
  cg.d = d;
  cg.M = (int)prio.size();
  std::vector<double> pv;
  for (const auto& kv : prio) {
    cg.lvl.insert(cg.lvl.end(), kv.first.begin(), kv.first.begin() + d);
    cg.idx.insert(cg.idx.end(), kv.first.begin() + d, kv.first.end());
    int t = 0;
    for (int n = 0; n < d; ++n) t += kv.first[n];
    cg.total.push_back(t);
    pv.push_back(kv.second);
  }
  std::vector<int> cand(cg.M);
  for (int i = 0; i < cg.M; ++i) cand[i] = i;
  std::sort(cand.begin(), cand.end(), [&](int a, int b) {
    if (pv[a] != pv[b]) return pv[a] > pv[b];
    return canon_less(cg, a, b);
  });
  const int take = std::min(room, cg.M);
  std::vector<int> chosen(cand.begin(), cand.begin() + take);
  std::sort(chosen.begin(), chosen.end(), [&](int a, int b) { return canon_less(cg, a, b); });
  if (take > max_new) return ENS_EINVAL;
  if (take > 0 && (!new_level_out || !new_index_out)) return ENS_EINVAL;
  for (int i = 0; i < take; ++i) {
    std::copy(cg.L(chosen[i]), cg.L(chosen[i]) + d, new_level_out + (size_t)i * d);
    std::copy(cg.K(chosen[i]), cg.K(chosen[i]) + d, new_index_out + (size_t)i * d);
  }
  *n_new_out = take;
  return ENS_OK;
}

int ens_group_variable(int32_t M, const double* pred, int32_t n_widths, const int32_t* widths,
                       const double* iter_seconds, int32_t* order_out, int32_t* group_width_out,
                       int32_t* group_count_out, int32_t* n_groups_out, double* cost_out) {
  if (M < 1 || !pred || !widths || !iter_seconds || !order_out || !group_width_out ||
      !group_count_out || !n_groups_out || !cost_out)
    return ENS_EINVAL;
  if (n_widths < 1 || n_widths > 64) return ENS_EINVAL;
  for (int w = 0; w < n_widths; ++w) {
    const int32_t s = widths[w];
    if (s < 1 || s > 64) return ENS_EINVAL;
    if (w > 0 && s <= widths[w - 1]) return ENS_EINVAL;
    if (!std::isfinite(iter_seconds[w]) || !(iter_seconds[w] > 0.0)) return ENS_EINVAL;
  }
  if (!finite_all(pred, (size_t)M)) return ENS_EINVAL;

  std::vector<int32_t> order(M);
  for (int i = 0; i < M; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    if (pred[a] != pred[b]) return pred[a] < pred[b];
    return a < b;
  });
  // best[i]: least predicted time of the first i samples of the order; the
  // last group ends at sample i - 1, whose prediction is the group's maximum
  std::vector<double> best(M + 1, 0.0);
  std::vector<int32_t> pick_w(M + 1, 0), pick_m(M + 1, 0);
  for (int i = 1; i <= M; ++i) {
    const double p = std::max(pred[order[i - 1]], 1.0);
    bool have = false;
    for (int w = 0; w < n_widths; ++w) {
      const double term = iter_seconds[w] * p;
      const int mmax = std::min(widths[w], i);
      for (int m = 1; m <= mmax; ++m) {
        const double v = best[i - m] + term;
        if (!have || v < best[i]) {
          best[i] = v;
          pick_w[i] = w;
          pick_m[i] = m;
          have = true;
        }
      }
    }
  }
  // walk back from the end, then emit the groups in ascending order
  std::vector<int32_t> gw, gc;
  for (int i = M; i > 0; i -= pick_m[i]) {
    gw.push_back(widths[pick_w[i]]);
    gc.push_back(pick_m[i]);
  }
  const int G = (int)gw.size();
  for (int g = 0; g < G; ++g) {
    group_width_out[g] = gw[G - 1 - g];
    group_count_out[g] = gc[G - 1 - g];
  }
  std::copy(order.begin(), order.end(), order_out);
  *n_groups_out = G;
  *cost_out = best[M];
  return ENS_OK;
}

}  // extern "C"
