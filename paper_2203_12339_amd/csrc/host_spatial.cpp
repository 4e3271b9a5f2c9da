// Spatial (output-side) compression of the truncated transport -- precompute
// Step 2 of Sec. 3.2 (Eq. 9, 10); CDF 9/7 per Sec. 5.
//
// Input: the Step-1 rows W_k^S in float64, row (p, k) holding its n_keep kept
// (column j, value) pairs, p in Morton order.  Per term k every column j of
// W_k^S is transformed along the output index p by w_1 (CDF 9/7, cdf97.h):
//   Z_k[:, j] = w_1 W_k^S[:, j]
// and the kept set S2(k) is the fewest entries of Z_k, largest |z| first
// (ties to the lower flat index u * n_cols + j), whose energy sum of z^2
// reaches the fraction tau of all of Z_k's energy (tau = 1 keeps every
// non-zero entry).
//
// Two passes over the columns, each on all host threads: the first bins
// every z^2 by the top bits of |z| (monotone in |z|) to find the bin where
// the running energy crosses tau; the second recomputes the columns, keeps
// the entries above that bin and ranks the ones inside it exactly.  The
// result is a CSR over the output coefficient u, entries of a row ordered by
// (k, j), with the term packed into the column word: (k << 24) | j.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "cdf97.h"
#include "host_internal.h"

namespace tlt {
namespace {

constexpr int KEY_SHIFT = 44;                     // 2^19 bins over positive doubles
constexpr size_t N_BINS = size_t(1) << (64 - KEY_SHIFT);

inline uint64_t bin_of(double z) {
  uint64_t b;
  const double a = std::fabs(z);
  std::memcpy(&b, &a, sizeof(b));
  return b >> KEY_SHIFT;
}

// one analysis level on x[0..n), result laid out [low | high] in x
void level_forward(double *x, double *t, int n) {
  auto step = [&](int parity, double c) {
    for (int i = parity; i < n; i += 2) x[i] += c * (x[cdf97::left_of(i)] + x[cdf97::right_of(i, n)]);
  };
  step(1, cdf97::A);
  step(0, cdf97::B);
  step(1, cdf97::G);
  step(0, cdf97::D);
  const int n_lo = (n + 1) / 2;
  for (int i = 0; i < n_lo; ++i) t[i] = x[2 * i] * cdf97::ZLO;
  for (int i = 0; i < n / 2; ++i) t[n_lo + i] = x[2 * i + 1] * cdf97::ZHI;
  std::memcpy(x, t, sizeof(double) * n);
}

struct Entry {
  int32_t u, j;
  double z;
};

// Column-major copy of one term's rows: entries of column j are
// (p, value) for p ascending.
struct Csc {
  std::vector<int64_t> ptr;
  std::vector<int32_t> row;
  std::vector<double> val;
};

void build_csc(int N, int n_cols, int K, int k, int64_t n_keep, const int32_t *col,
               const double *val, Csc &c) {
  c.ptr.assign((size_t)n_cols + 1, 0);
  for (int p = 0; p < N; ++p) {
    const size_t off = ((size_t)p * K + k) * (size_t)n_keep;
    for (int64_t t = 0; t < n_keep; ++t) ++c.ptr[(size_t)col[off + t] + 1];
  }
  for (int j = 0; j < n_cols; ++j) c.ptr[j + 1] += c.ptr[j];
  c.row.resize(c.ptr[n_cols]);
  c.val.resize(c.ptr[n_cols]);
  std::vector<int64_t> cur(c.ptr.begin(), c.ptr.end() - 1);
  for (int p = 0; p < N; ++p) {
    const size_t off = ((size_t)p * K + k) * (size_t)n_keep;
    for (int64_t t = 0; t < n_keep; ++t) {
      const int64_t d = cur[col[off + t]]++;
      c.row[d] = p;
      c.val[d] = val[off + t];
    }
  }
}

template <typename F>
void for_threads(int n_threads, F &&f) {
  std::vector<std::thread> th;
  for (int t = 1; t < n_threads; ++t) th.emplace_back(f, t);
  f(0);
  for (auto &x : th) x.join();
}

// One synthesis level on x[0..n) from [low | high], evaluated on the
// interleaved window [lo, hi) only: t must be zero outside the window (the
// lifting steps read one neighbour on each side), and is zero again on
// return; x[lo, hi) receives the result.
void level_inverse(double *x, double *t, int n, int lo, int hi) {
  const int n_lo = (n + 1) / 2;
  for (int i = lo; i < hi; ++i) t[i] = (i & 1) ? x[n_lo + (i >> 1)] / cdf97::ZHI : x[i >> 1] / cdf97::ZLO;
  auto step = [&](int parity, double c) {
    for (int i = lo + ((lo & 1) != parity); i < hi; i += 2)
      t[i] -= c * (t[cdf97::left_of(i)] + t[cdf97::right_of(i, n)]);
  };
  step(0, cdf97::D);
  step(1, cdf97::G);
  step(0, cdf97::B);
  step(1, cdf97::A);
  for (int i = lo; i < hi; ++i) {
    x[i] = t[i];
    t[i] = 0.0;
  }
}

}  // namespace

void synthesis_build(int N, const std::vector<int> &sizes, int n_threads, std::vector<int32_t> &rowptr,
                     std::vector<int32_t> &col, std::vector<double> &w) {
  // Column u of w_1^{-1} is the synthesis of the unit coefficient u.  Its
  // non-zero range is tracked level by level: a level's interleave maps the
  // band entries in range to their positions, and its four lifting steps
  // widen that by at most one position each, so only that window is
  // computed (the rest of the level's output is exactly zero).
  const int L = (int)sizes.size();
  n_threads = std::max(1, std::min(n_threads, 64));
  std::vector<std::vector<std::pair<int32_t, double>>> cols(N);   // (o, weight) per u
  for_threads(n_threads, [&](int th) {
    std::vector<double> x(N, 0.0), t(N, 0.0);
    const int u0 = (int)((int64_t)N * th / n_threads), u1 = (int)((int64_t)N * (th + 1) / n_threads);
    for (int u = u0; u < u1; ++u) {
      x[u] = 1.0;
      int lo = u, hi = u + 1;               // x is zero outside [lo, hi)
      for (int lv = L - 1; lv >= 0; --lv) {
        const int n = sizes[lv], n_lo = (n + 1) / 2;
        if (lo >= n) continue;              // this level sees only zeros
        const int h = std::min(hi, n);
        int a = n, b = -1;                  // interleaved positions of [lo, h)
        if (lo < n_lo) {
          a = std::min(a, 2 * lo);
          b = std::max(b, 2 * (std::min(h, n_lo) - 1));
        }
        if (h > n_lo) {
          a = std::min(a, 2 * (std::max(lo, n_lo) - n_lo) + 1);
          b = std::max(b, 2 * (h - 1 - n_lo) + 1);
        }
        const int wlo = std::max(0, a - 4), whi = std::min(n, b + 5);
        level_inverse(x.data(), t.data(), n, wlo, whi);
        for (int i = lo; i < std::min(h, wlo); ++i) x[i] = 0.0;     // band entries consumed
        for (int i = std::max(lo, whi); i < h; ++i) x[i] = 0.0;
        lo = wlo;
        hi = hi > n ? hi : whi;
      }
      for (int o = lo; o < hi; ++o) {
        if (x[o] != 0.0) cols[u].push_back({o, x[o]});
        x[o] = 0.0;
      }
    }
  });
  rowptr.assign((size_t)N + 1, 0);
  for (int u = 0; u < N; ++u)
    for (auto &e : cols[u]) ++rowptr[e.first + 1];
  for (int o = 0; o < N; ++o) rowptr[o + 1] += rowptr[o];
  col.resize(rowptr[N]);
  w.resize(rowptr[N]);
  std::vector<int32_t> cur(rowptr.begin(), rowptr.end() - 1);
  for (int u = 0; u < N; ++u)
    for (auto &e : cols[u]) {
      const int32_t d = cur[e.first]++;
      col[d] = u;
      w[d] = e.second;
    }
}

std::vector<int> cdf97_sizes(int n, int levels) {
  std::vector<int> s;
  while (n >= cdf97::MIN_SPLIT && (levels == 0 || (int)s.size() < levels)) {
    s.push_back(n);
    n = (n + 1) / 2;
  }
  return s;
}

tlt_status spatial_build(int N, int n_cols, int K, int64_t n_keep, const int32_t *col,
                         const double *val, double energy, int levels, int n_threads,
                         SpatialCsr &out, std::string *err) {
  if (N < cdf97::MIN_SPLIT) return fail(err, TLT_E_ARG, "spatial compression needs N >= 8");
  if (!(energy > 0.0 && energy <= 1.0)) return fail(err, TLT_E_ARG, "energy must be in (0, 1]");
  if (levels < 0 || levels > cdf97::MAX_LEVELS) return fail(err, TLT_E_ARG, "levels out of range");
  if (K < 1 || K > 127 || n_cols < 1 || n_cols >= (1 << 24) || n_keep < 1 || n_keep > n_cols)
    return fail(err, TLT_E_ARG, "spatial compression supports K <= 127 and n_cols < 2^24");
  out.sizes = cdf97_sizes(N, levels);
  if (levels > 0 && (int)out.sizes.size() < levels)
    return fail(err, TLT_E_ARG, "too many levels for this vertex count");
  for (size_t i = 0; i < (size_t)N * K * n_keep; ++i)
    if (col[i] < 0 || col[i] >= n_cols) return fail(err, TLT_E_FORMAT, "column out of range");
  n_threads = std::max(1, std::min(n_threads, 64));
  const bool keep_all = energy >= 1.0;

  std::vector<std::vector<Entry>> kept_k(K);     // per term, grouped by thread then j
  out.nnz_k.assign(K, 0);
  out.energy_kept.assign(K, 0.0);
  Csc csc;
  for (int k = 0; k < K; ++k) {
    build_csc(N, n_cols, K, k, n_keep, col, val, csc);
    // transform column j into x (dense, N entries)
    auto column = [&](int j, std::vector<double> &x, std::vector<double> &t) -> bool {
      const int64_t a = csc.ptr[j], b = csc.ptr[j + 1];
      if (a == b) return false;
      std::fill(x.begin(), x.end(), 0.0);
      for (int64_t e = a; e < b; ++e) x[csc.row[e]] = csc.val[e];
      for (int n : out.sizes) level_forward(x.data(), t.data(), n);
      return true;
    };
    auto j_range = [&](int t) {
      const int64_t j0 = (int64_t)n_cols * t / n_threads, j1 = (int64_t)n_cols * (t + 1) / n_threads;
      return std::make_pair((int)j0, (int)j1);
    };
    // pass 1: energy per magnitude bin
    uint64_t cut_bin = 0;
    double e_above = 0.0, total = 0.0, target = 0.0;
    if (!keep_all) {
      std::vector<std::vector<double>> hist(n_threads);
      for_threads(n_threads, [&](int t) {
        std::vector<double> x(N), tmp(N);
        hist[t].assign(N_BINS, 0.0);
        auto [j0, j1] = j_range(t);
        for (int j = j0; j < j1; ++j) {
          if (!column(j, x, tmp)) continue;
          for (int u = 0; u < N; ++u)
            if (x[u] != 0.0) hist[t][bin_of(x[u])] += x[u] * x[u];
        }
      });
      std::vector<double> h(N_BINS, 0.0);
      for (int t = 0; t < n_threads; ++t)
        for (size_t b = 0; b < N_BINS; ++b) h[b] += hist[t][b];
      hist.clear();
      for (size_t b = N_BINS; b-- > 0;) total += h[b];
      target = energy * total;
      // the bin in which the running energy (largest first) reaches tau
      double run = 0.0;
      bool found = false;
      uint64_t last = 0;
      for (size_t b = N_BINS; b-- > 0;) {
        if (h[b] == 0.0) continue;
        last = b;
        if (run + h[b] >= target) {
          cut_bin = b;
          found = true;
          break;
        }
        run += h[b];
      }
      if (!found) {              // rounding left tau * total above the sum
        cut_bin = last;
        run -= h[last];
      }
      e_above = run;
    }
    // pass 2: entries above the cut bin, and the candidates inside it
    std::vector<std::vector<Entry>> above(n_threads), inside(n_threads);
    for_threads(n_threads, [&](int t) {
      std::vector<double> x(N), tmp(N);
      auto [j0, j1] = j_range(t);
      for (int j = j0; j < j1; ++j) {
        if (!column(j, x, tmp)) continue;
        for (int u = 0; u < N; ++u) {
          const double z = x[u];
          if (z == 0.0) continue;
          if (keep_all) {
            above[t].push_back({u, j, z});
            continue;
          }
          const uint64_t b = bin_of(z);
          if (b > cut_bin) above[t].push_back({u, j, z});
          else if (b == cut_bin) inside[t].push_back({u, j, z});
        }
      }
    });
    std::vector<Entry> &kk = kept_k[k];
    double e_kept = 0.0;
    for (int t = 0; t < n_threads; ++t) {
      for (const Entry &e : above[t]) e_kept += e.z * e.z;
      kk.insert(kk.end(), above[t].begin(), above[t].end());
      std::vector<Entry>().swap(above[t]);
    }
    if (!keep_all) {
      std::vector<Entry> cand;
      for (int t = 0; t < n_threads; ++t) cand.insert(cand.end(), inside[t].begin(), inside[t].end());
      std::sort(cand.begin(), cand.end(), [&](const Entry &a, const Entry &b) {
        const double fa = std::fabs(a.z), fb = std::fabs(b.z);
        if (fa != fb) return fa > fb;
        const int64_t ia = (int64_t)a.u * n_cols + a.j, ib = (int64_t)b.u * n_cols + b.j;
        return ia < ib;
      });
      double run = e_above;
      std::vector<Entry> take;
      for (const Entry &e : cand) {
        if (run >= target) break;
        run += e.z * e.z;
        take.push_back(e);
        e_kept += e.z * e.z;
      }
      // keep the per-row (k, j) order: merge the ranked candidates back by j
      kk.insert(kk.end(), take.begin(), take.end());
      std::stable_sort(kk.begin(), kk.end(), [](const Entry &a, const Entry &b) { return a.j < b.j; });
      out.energy_kept[k] = total > 0.0 ? e_kept / total : 1.0;
    } else {
      out.energy_kept[k] = 1.0;
    }
    out.nnz_k[k] = (int64_t)kk.size();
  }
  // CSR over u, entries of a row in (k, j) order
  out.rowptr.assign((size_t)N + 1, 0);
  for (int k = 0; k < K; ++k)
    for (const Entry &e : kept_k[k]) ++out.rowptr[(size_t)e.u + 1];
  for (int u = 0; u < N; ++u) out.rowptr[u + 1] += out.rowptr[u];
  const int64_t nnz = out.rowptr[N];
  out.col.resize(nnz);
  out.val.resize(nnz);
  std::vector<int64_t> cur(out.rowptr.begin(), out.rowptr.end() - 1);
  for (int k = 0; k < K; ++k) {
    for (const Entry &e : kept_k[k]) {
      const int64_t d = cur[e.u]++;
      out.col[d] = ((uint32_t)k << 24) | (uint32_t)e.j;
      out.val[d] = e.z;
    }
    std::vector<Entry>().swap(kept_k[k]);
  }
  return TLT_OK;
}

}  // namespace tlt

extern "C" tlt_status tlt_spatial_rows(int32_t n_vertices, int32_t n_cols, int32_t K, int64_t n_keep,
                                       const int32_t *col, const double *val, double energy,
                                       int32_t levels, int64_t *rowptr_out, uint32_t *col_out,
                                       double *val_out, int64_t capacity) {
  using namespace tlt;
  if (n_vertices < 1 || !col || !val || !rowptr_out) return fail(nullptr, TLT_E_ARG, "bad arguments");
  SpatialCsr csr;
  const unsigned hw = std::max(1u, std::min(std::thread::hardware_concurrency(), 16u));
  const tlt_status s = spatial_build(n_vertices, n_cols, K, n_keep, col, val, energy, levels,
                                     (int)hw, csr, nullptr);
  if (s != TLT_OK) return s;
  std::memcpy(rowptr_out, csr.rowptr.data(), sizeof(int64_t) * ((size_t)n_vertices + 1));
  const int64_t nnz = csr.rowptr[n_vertices];
  if (nnz > capacity) return fail(nullptr, TLT_E_ARG, "capacity below the kept entries");
  if (nnz > 0 && (!col_out || !val_out)) return fail(nullptr, TLT_E_ARG, "NULL output");
  if (nnz > 0) {
    std::memcpy(col_out, csr.col.data(), sizeof(uint32_t) * nnz);
    std::memcpy(val_out, csr.val.data(), sizeof(double) * nnz);
  }
  return TLT_OK;
}

extern "C" tlt_status tlt_spatial_synthesis(int32_t n_vertices, int32_t levels, int32_t *rowptr_out,
                                            int32_t *col_out, double *w_out, int64_t capacity) {
  using namespace tlt;
  if (n_vertices < cdf97::MIN_SPLIT || levels < 0 || levels > cdf97::MAX_LEVELS || !rowptr_out)
    return fail(nullptr, TLT_E_ARG, "bad arguments");
  const std::vector<int> sizes = cdf97_sizes(n_vertices, levels);
  if (levels > 0 && (int)sizes.size() < levels) return fail(nullptr, TLT_E_ARG, "too many levels");
  std::vector<int32_t> rp, col;
  std::vector<double> w;
  const unsigned hw = std::max(1u, std::min(std::thread::hardware_concurrency(), 16u));
  synthesis_build(n_vertices, sizes, (int)hw, rp, col, w);
  std::memcpy(rowptr_out, rp.data(), sizeof(int32_t) * ((size_t)n_vertices + 1));
  const int64_t nnz = rp[n_vertices];
  if (nnz > capacity) return fail(nullptr, TLT_E_ARG, "capacity below the operator's entries");
  if (nnz > 0 && (!col_out || !w_out)) return fail(nullptr, TLT_E_ARG, "NULL output");
  std::memcpy(col_out, col.data(), sizeof(int32_t) * nnz);
  std::memcpy(w_out, w.data(), sizeof(double) * nnz);
  return TLT_OK;
}
