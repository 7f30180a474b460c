// Aggregation-based algebraic multigrid hierarchy for the coarse system
// (Section 4.1, "Algebraic multigrid"): host set-up.  The paper names the
// ingredients (unsmoothed aggregation on the order-1 matrix, a recursive
// K-cycle, damped Jacobi); the readings fixed here:
//   * unknowns: the free vertices in ascending vertex id;
//   * strong couplings of row i: j != i with a_ij < 0 and -a_ij >= 0.25 max_k(-a_ik);
//   * one coarsening step = two pairwise passes: rows visited in order, an
//     unmatched row takes the unmatched strong neighbour with the most
//     negative coupling (ties: smallest index) or stays alone; aggregates are
//     numbered in order of creation; the second pass runs on the Galerkin
//     matrix of the first, so aggregates hold at most 4 unknowns;
//   * Galerkin coarse matrices P^T A P with P the 0/1 aggregate indicator;
//   * coarsening stops at 400 unknowns or less, or when a step keeps more
//     than two thirds of them; the coarsest matrix is inverted densely.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "sem_internal.h"

namespace sem {

namespace {

constexpr double kStrong = 0.25;
constexpr int64_t kCoarsest = 400;

struct Csr {
  int64_t n = 0;
  std::vector<int32_t> off, col;
  std::vector<double> val;
};

// aggregate id of every row, one pairwise pass
std::vector<int32_t> pairwise(const Csr& A, int32_t& nagg) {
  std::vector<int32_t> agg(A.n, -1);
  nagg = 0;
  for (int64_t i = 0; i < A.n; ++i) {
    if (agg[i] >= 0) continue;
    double s = 0.0;
    bool any = false;
    for (int32_t q = A.off[i]; q < A.off[i + 1]; ++q)
      if (A.col[q] != i && A.val[q] < 0.0) {
        s = any ? std::max(s, -A.val[q]) : -A.val[q];
        any = true;
      }
    const double thr = kStrong * s;
    double best = 0.0;
    int64_t bj = -1;
    if (any)
      for (int32_t q = A.off[i]; q < A.off[i + 1]; ++q) {
        const int64_t j = A.col[q];
        const double a = A.val[q];
        if (j == i || !(a < 0.0) || !(-a >= thr) || agg[j] >= 0) continue;
        if (bj < 0 || a < best || (a == best && j < bj)) {
          best = a;
          bj = j;
        }
      }
    agg[i] = nagg;
    if (bj >= 0) agg[bj] = nagg;
    ++nagg;
  }
  return agg;
}

// P^T A P for the aggregate map agg (nc aggregates); columns sorted
Csr galerkin(const Csr& A, const std::vector<int32_t>& agg, int32_t nc) {
  std::vector<std::vector<std::pair<int32_t, double>>> rows(nc);
  for (int64_t i = 0; i < A.n; ++i)
    for (int32_t q = A.off[i]; q < A.off[i + 1]; ++q) rows[agg[i]].push_back({agg[A.col[q]], A.val[q]});
  Csr C;
  C.n = nc;
  C.off.assign(nc + 1, 0);
  for (int32_t r = 0; r < nc; ++r) {
    auto& l = rows[r];
    std::stable_sort(l.begin(), l.end(), [](auto& x, auto& y) { return x.first < y.first; });
    for (size_t q = 0; q < l.size(); ++q) {
      if (q > 0 && l[q].first == l[q - 1].first)
        C.val.back() += l[q].second;
      else {
        C.col.push_back(l[q].first);
        C.val.push_back(l[q].second);
      }
    }
    C.off[r + 1] = (int32_t)C.col.size();
  }
  return C;
}

// dense inverse of an SPD matrix by Cholesky (row-major)
std::vector<double> spd_inverse(const Csr& A) {
  const int64_t n = A.n;
  std::vector<double> M((size_t)n * n, 0.0), L((size_t)n * n, 0.0), Inv((size_t)n * n, 0.0);
  for (int64_t i = 0; i < n; ++i)
    for (int32_t q = A.off[i]; q < A.off[i + 1]; ++q) M[i * n + A.col[q]] += A.val[q];
  for (int64_t j = 0; j < n; ++j) {
    double d = M[j * n + j];
    for (int64_t k = 0; k < j; ++k) d -= L[j * n + k] * L[j * n + k];
    if (!(d > 0.0)) throw Error{SEM_EMESH, "coarsest AMG matrix not positive definite"};
    L[j * n + j] = std::sqrt(d);
    for (int64_t i = j + 1; i < n; ++i) {
      double v = M[i * n + j];
      for (int64_t k = 0; k < j; ++k) v -= L[i * n + k] * L[j * n + k];
      L[i * n + j] = v / L[j * n + j];
    }
  }
  // columns of the inverse: solve L L^T x = e_c
  std::vector<double> y(n);
  for (int64_t c = 0; c < n; ++c) {
    for (int64_t i = 0; i < n; ++i) {
      double v = i == c ? 1.0 : 0.0;
      for (int64_t k = 0; k < i; ++k) v -= L[i * n + k] * y[k];
      y[i] = v / L[i * n + i];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      double v = y[i];
      for (int64_t k = i + 1; k < n; ++k) v -= L[k * n + i] * Inv[k * n + c];
      Inv[i * n + c] = v / L[i * n + i];
    }
  }
  return Inv;
}

}  // namespace

void build_amg(const HostTables& T, AmgHierarchy& H) {
  H = AmgHierarchy{};
  // level 0: the free vertices in ascending vertex id
  const int64_t nc = T.nc;
  H.nd_of.resize(nc);
  std::vector<int32_t> pos(nc, -1);  // coarse (nested-dissection) index -> level-0 index
  {
    int32_t q = 0;
    for (int64_t v = 0; v < T.V; ++v)
      if (T.cidx[v] >= 0) {
        H.nd_of[q] = T.cidx[v];
        pos[T.cidx[v]] = q;
        ++q;
      }
  }
  Csr A;
  A.n = nc;
  A.off.assign(nc + 1, 0);
  for (int64_t q = 0; q < nc; ++q) {
    const int32_t r = H.nd_of[q];
    std::vector<std::pair<int32_t, double>> row;
    for (int32_t k = T.ac_off[r]; k < T.ac_off[r + 1]; ++k) row.push_back({pos[T.ac_col[k]], T.ac_val[k]});
    std::sort(row.begin(), row.end(), [](auto& x, auto& y) { return x.first < y.first; });
    for (auto& e : row) {
      A.col.push_back(e.first);
      A.val.push_back(e.second);
    }
    A.off[q + 1] = (int32_t)A.col.size();
  }
  while (true) {
    AmgLevel lv;
    lv.n = A.n;
    lv.off = A.off;
    lv.col = A.col;
    lv.val = A.val;
    lv.diag.assign(A.n, 0.0);
    for (int64_t i = 0; i < A.n; ++i)
      for (int32_t q = A.off[i]; q < A.off[i + 1]; ++q)
        if (A.col[q] == i) lv.diag[i] += A.val[q];
    if (A.n <= kCoarsest) {
      H.levels.push_back(std::move(lv));
      break;
    }
    int32_t n1 = 0, n2 = 0;
    const std::vector<int32_t> a1 = pairwise(A, n1);
    const Csr A1 = galerkin(A, a1, n1);
    const std::vector<int32_t> a2 = pairwise(A1, n2);
    if ((int64_t)n2 > (2 * A.n) / 3) {
      H.levels.push_back(std::move(lv));
      break;
    }
    lv.agg.resize(A.n);
    for (int64_t i = 0; i < A.n; ++i) lv.agg[i] = a2[a1[i]];
    // members of each aggregate, ascending (restriction sums them in this order)
    lv.moff.assign(n2 + 1, 0);
    for (int64_t i = 0; i < A.n; ++i) ++lv.moff[lv.agg[i] + 1];
    for (int32_t a = 0; a < n2; ++a) lv.moff[a + 1] += lv.moff[a];
    lv.mem.resize(A.n);
    std::vector<int32_t> fill(lv.moff.begin(), lv.moff.end() - 1);
    for (int64_t i = 0; i < A.n; ++i) lv.mem[fill[lv.agg[i]]++] = (int32_t)i;
    Csr Ac = galerkin(A, lv.agg, n2);
    H.levels.push_back(std::move(lv));
    A = std::move(Ac);
  }
  Csr last;
  const AmgLevel& L = H.levels.back();
  last.n = L.n;
  last.off = L.off;
  last.col = L.col;
  last.val = L.val;
  H.coarse_inv = last.n > 0 ? spd_inverse(last) : std::vector<double>{};
}

}  // namespace sem
