// Performance-aware submatrix combination (paper, Sec. IV-B, Eq. 9 and Eq. 10).
//
// Host code.  Groups of molecules share one submatrix, whose rows are the union of
// the rows of their block columns.  Two groups whose submatrices share rows are
// candidates; combining them replaces two submatrices of dimensions n_i, n_j by one
// of dimension n_i + n_j - n_ij (n_ij: the functions of the shared rows).  The gain
// cost(n_i) + cost(n_j) - cost(n_i + n_j - n_ij) is positive exactly when the
// criterion holds: Eq. 9 compares the cubic flop counts, Eq. 10 the predicted run
// times n^3 / rate(n) from the measured GEMM throughput.  The candidate pair with the
// largest gain is combined first (ties: the pair whose smallest molecules come first
// in lexicographic order) until no candidate pair gains.
//
// A max-heap holds the gain of every candidate pair; combining two groups retires
// both (their heap entries become stale by version) and pushes the pairs of the new
// group, found through an index from each row molecule to the groups containing it.
#include <algorithm>
#include <cmath>
#include <queue>
#include <string>
#include <vector>

#include "common.h"

namespace nolsm {

struct RateTable {
  const double *n = nullptr, *r = nullptr;
  int np = 0;
  // linear interpolation, clamped at the ends (separate statements: no fused
  // multiply-add, so the result is the same in any IEEE double implementation)
  double at(double x) const {
    if (x <= n[0]) return r[0];
    if (x >= n[np - 1]) return r[np - 1];
    int i = 0;
    while (n[i + 1] < x) ++i;
    const double t = (x - n[i]) / (n[i + 1] - n[i]);
    const double d = (r[i + 1] - r[i]) * t;
    return r[i] + d;
  }
};

// Gains compared as exact integers (Eq. 9) or doubles (Eq. 10).
struct Gain {
  __int128 i = 0;
  double f = 0.0;
};

struct CombineState {
  int criterion = 9;
  int max_n = 0;
  RateTable table;
  const int32_t *dims = nullptr;

  Gain cost(int64_t n) const {
    Gain g;
    if (criterion == 9) {
      g.i = (__int128)n * n * n;
    } else {
      const double n3 = (double)n * (double)n * (double)n;
      g.f = n3 / table.at((double)n);
    }
    return g;
  }
  // gain of combining: cost(a) + cost(b) - cost(u), in the oracle's order of operations
  Gain gain(int64_t na, int64_t nb, int64_t nu) const {
    const Gain a = cost(na), b = cost(nb), u = cost(nu);
    Gain g;
    if (criterion == 9) {
      g.i = a.i + b.i - u.i;
    } else {
      const double s = a.f + b.f;
      g.f = s - u.f;
    }
    return g;
  }
  bool positive(const Gain &g) const { return criterion == 9 ? g.i > 0 : g.f > 0.0; }
  bool greater(const Gain &x, const Gain &y) const {
    return criterion == 9 ? x.i > y.i : x.f > y.f;
  }
};

struct Cand {
  Gain g;
  int32_t ka, kb;       // group keys (smallest molecules), ka < kb
  int32_t a, b;         // group slots
  uint32_t va, vb;      // versions when pushed
};

}  // namespace nolsm

using namespace nolsm;

namespace nolsm {
nolsm_status set_error(nolsm_status code, const char *msg);   // nolsm_last_error() text
}

extern "C" nolsm_status nolsm_combine(const nolsm_pattern *pat, const int32_t *mols, int32_t K,
                                      const nolsm_combine_options *opt, int32_t *grp_ptr,
                                      int32_t *grp_mols, int32_t *ngroups_out) {
  if (!pat || !opt || !grp_ptr || !ngroups_out || K < 0 || (K > 0 && (!mols || !grp_mols)))
    return set_error(NOLSM_EINVAL, "nolsm_combine: null argument or K < 0");
  if (!pat->blk_dim || !pat->colptr || !pat->rowblk)
    return set_error(NOLSM_EINVAL, "nolsm_combine: pattern arrays must be set (host copies)");
  CombineState cs;
  cs.criterion = opt->criterion;
  cs.max_n = opt->max_n;
  cs.dims = pat->blk_dim;
  if (cs.criterion != 9 && cs.criterion != 10)
    return set_error(NOLSM_EINVAL, "nolsm_combine: criterion must be 9 or 10");
  if (cs.max_n < 0) return set_error(NOLSM_EINVAL, "nolsm_combine: max_n must be >= 0");
  if (cs.criterion == 10) {
    if (opt->npoints < 1 || !opt->rate_n || !opt->rate)
      return set_error(NOLSM_EINVAL, "nolsm_combine: criterion 10 needs a rate table");
    for (int i = 0; i < opt->npoints; ++i) {
      if (!(opt->rate[i] > 0.0) || !std::isfinite(opt->rate[i]) || !std::isfinite(opt->rate_n[i]) ||
          (i > 0 && !(opt->rate_n[i] > opt->rate_n[i - 1])))
        return set_error(NOLSM_EINVAL,
                         "nolsm_combine: rate table needs ascending dimensions and positive rates");
    }
    cs.table.n = opt->rate_n;
    cs.table.r = opt->rate;
    cs.table.np = opt->npoints;
  }
  const int nmol = pat->nmol;
  std::vector<int32_t> slot_of(nmol, -1);
  for (int i = 0; i < K; ++i) {
    if (mols[i] < 0 || mols[i] >= nmol || slot_of[mols[i]] >= 0)
      return set_error(NOLSM_EINVAL, "nolsm_combine: molecule out of range or repeated");
    slot_of[mols[i]] = i;
  }
  // groups live in slots 0..K-1; a combined group keeps the slot of the smaller key
  std::vector<std::vector<int32_t>> rows(K), members(K);
  std::vector<int64_t> nrow(K);
  std::vector<int32_t> key(K);
  std::vector<uint32_t> ver(K, 0);
  std::vector<char> alive(K, 1);
  std::vector<std::vector<int32_t>> row_groups(nmol);   // row molecule -> slots containing it
  for (int i = 0; i < K; ++i) {
    const int k = mols[i];
    key[i] = k;
    members[i] = {k};
    for (int64_t t = pat->colptr[k]; t < pat->colptr[k + 1]; ++t) rows[i].push_back(pat->rowblk[t]);
    std::sort(rows[i].begin(), rows[i].end());
    rows[i].erase(std::unique(rows[i].begin(), rows[i].end()), rows[i].end());
    nrow[i] = 0;
    for (const int j : rows[i]) {
      nrow[i] += pat->blk_dim[j];
      row_groups[j].push_back(i);
    }
  }
  auto shared_dim = [&](int a, int b) {
    int64_t s = 0;
    size_t x = 0, y = 0;
    const std::vector<int32_t> &ra = rows[a], &rb = rows[b];
    while (x < ra.size() && y < rb.size()) {
      if (ra[x] < rb[y]) ++x;
      else if (rb[y] < ra[x]) ++y;
      else { s += pat->blk_dim[ra[x]]; ++x; ++y; }
    }
    return s;
  };
  auto worse = [&](const Cand &x, const Cand &y) {     // heap order: y comes first
    if (cs.greater(y.g, x.g)) return true;
    if (cs.greater(x.g, y.g)) return false;
    if (x.ka != y.ka) return x.ka > y.ka;
    return x.kb > y.kb;
  };
  std::priority_queue<Cand, std::vector<Cand>, decltype(worse)> heap(worse);
  std::vector<uint32_t> stamp(K, 0);
  uint32_t tick = 0;
  auto push_pairs = [&](int a) {
    ++tick;
    stamp[a] = tick;
    for (const int j : rows[a])
      for (const int b : row_groups[j]) {
        if (!alive[b] || stamp[b] == tick) continue;
        stamp[b] = tick;
        const int64_t nu = nrow[a] + nrow[b] - shared_dim(a, b);
        if (cs.max_n > 0 && nu > cs.max_n) continue;
        Cand c;
        c.g = cs.gain(nrow[a], nrow[b], nu);
        if (!cs.positive(c.g)) continue;
        const bool af = key[a] < key[b];
        c.a = af ? a : b;
        c.b = af ? b : a;
        c.ka = key[c.a];
        c.kb = key[c.b];
        c.va = ver[c.a];
        c.vb = ver[c.b];
        heap.push(c);
      }
  };
  // initial pairs: each pushed once, from the slot with the smaller key
  for (int a = 0; a < K; ++a) {
    ++tick;
    stamp[a] = tick;
    for (const int j : rows[a])
      for (const int b : row_groups[j]) {
        if (stamp[b] == tick) continue;
        stamp[b] = tick;
        if (key[b] < key[a]) continue;
        const int64_t nu = nrow[a] + nrow[b] - shared_dim(a, b);
        if (cs.max_n > 0 && nu > cs.max_n) continue;
        Cand c;
        c.g = cs.gain(nrow[a], nrow[b], nu);
        if (!cs.positive(c.g)) continue;
        c.a = a;
        c.b = b;
        c.ka = key[a];
        c.kb = key[b];
        c.va = ver[a];
        c.vb = ver[b];
        heap.push(c);
      }
  }
  while (!heap.empty()) {
    const Cand c = heap.top();
    heap.pop();
    if (!alive[c.a] || !alive[c.b] || ver[c.a] != c.va || ver[c.b] != c.vb) continue;
    const int a = c.a, b = c.b;                  // key[a] < key[b]: a keeps the group
    std::vector<int32_t> u;
    u.reserve(rows[a].size() + rows[b].size());
    std::set_union(rows[a].begin(), rows[a].end(), rows[b].begin(), rows[b].end(),
                   std::back_inserter(u));
    for (const int j : rows[b]) {
      std::vector<int32_t> &lst = row_groups[j];
      lst.erase(std::remove(lst.begin(), lst.end(), b), lst.end());
      if (!std::binary_search(rows[a].begin(), rows[a].end(), j)) lst.push_back(a);
    }
    rows[a].swap(u);
    nrow[a] = 0;
    for (const int j : rows[a]) nrow[a] += pat->blk_dim[j];
    members[a].insert(members[a].end(), members[b].begin(), members[b].end());
    std::sort(members[a].begin(), members[a].end());
    alive[b] = 0;
    rows[b].clear();
    members[b].clear();
    ++ver[a];
    ++ver[b];
    push_pairs(a);
  }
  // output ordered by first molecule
  std::vector<int> order;
  for (int i = 0; i < K; ++i)
    if (alive[i]) order.push_back(i);
  std::sort(order.begin(), order.end(), [&](int x, int y) { return key[x] < key[y]; });
  int pos = 0, g = 0;
  grp_ptr[0] = 0;
  for (const int i : order) {
    for (const int k : members[i]) grp_mols[pos++] = k;
    grp_ptr[++g] = pos;
  }
  *ngroups_out = g;
  return NOLSM_OK;
}
