// Host-side precompute of the translucent-transport library.
//
// * tlt_prepare_scene: geometry and material-basis precompute (float64).
// * tlt_host_build_rows: the transport rows of precompute Step 1 (Sec. 3.2):
//   for every output vertex o and basis term k the kernel row
//   btilde_k(|x_o - x_i|) over the Morton-ordered vertices, its orthonormal
//   Haar transform (Eq. 8), and the n_keep coefficients of largest magnitude.
//   Runs on all host cores (std::thread), float64 throughout.
//
// This is offline load-time work; nothing here runs per frame.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tlt.h"
#include "host_internal.h"

namespace tlt {

thread_local std::string g_thread_error;

tlt_status fail(std::string *dst, tlt_status st, const std::string &msg) {
  if (dst) *dst = msg;
  g_thread_error = msg;
  return st;
}

// ---------------------------------------------------------------------------
// Morton order
// ---------------------------------------------------------------------------

static void morton_perm(int n, const double *v, int32_t *perm) {
  double lo[3], hi[3];
  for (int a = 0; a < 3; ++a) { lo[a] = v[a]; hi[a] = v[a]; }
  for (int i = 1; i < n; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], v[3 * i + a]);
      hi[a] = std::max(hi[a], v[3 * i + a]);
    }
  const double scale = double(1u << 21);
  std::vector<uint64_t> key(n);
  for (int i = 0; i < n; ++i) {
    uint64_t q[3];
    for (int a = 0; a < 3; ++a) {
      double t = (v[3 * i + a] - lo[a]) / (hi[a] - lo[a]);
      t = std::floor(t * scale);
      if (!(t >= 0.0)) t = 0.0;             // degenerate extent -> 0
      if (t > scale - 1.0) t = scale - 1.0;
      q[a] = (uint64_t)t;
    }
    uint64_t k = 0;
    for (int b = 0; b < 21; ++b) {
      k |= ((q[0] >> b) & 1ull) << (3 * b + 2);
      k |= ((q[1] >> b) & 1ull) << (3 * b + 1);
      k |= ((q[2] >> b) & 1ull) << (3 * b);
    }
    key[i] = k;
  }
  std::vector<int32_t> idx(n);
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(),
                   [&](int32_t a, int32_t b) { return key[a] < key[b]; });
  std::memcpy(perm, idx.data(), sizeof(int32_t) * n);
}

// ---------------------------------------------------------------------------
// Real SH (no Condon-Shortley phase) and the clamped-cosine transfer.
// ---------------------------------------------------------------------------

static double clamped_cosine_coeff(int l) {
  // 2 pi int_0^1 t P_l(t) dt in closed form.
  const double pi = M_PI;
  if (l == 0) return pi;
  if (l == 1) return 2.0 * pi / 3.0;
  if (l % 2 == 1) return 0.0;
  double fact_l = 1.0, fact_h = 1.0;
  for (int i = 2; i <= l; ++i) fact_l *= i;
  for (int i = 2; i <= l / 2; ++i) fact_h *= i;
  double sgn = ((l / 2 - 1) % 2 == 0) ? 1.0 : -1.0;
  return 2.0 * pi * sgn / double((l + 2) * (l - 1)) * fact_l /
         (std::ldexp(1.0, l) * fact_h * fact_h);
}

static void real_sh(int lmax, const double *d, double *out) {
  const double x = d[0], y = d[1], z = d[2];
  // Pt[l][m] = P_l^m(z) / sin^m(theta)
  double P[8][8];
  for (int m = 0; m <= lmax; ++m) {
    double df = 1.0;
    for (int k = 1; k < 2 * m; k += 2) df *= k;
    P[m][m] = df;
    if (m + 1 <= lmax) P[m + 1][m] = z * (2 * m + 1) * P[m][m];
    for (int l = m + 2; l <= lmax; ++l)
      P[l][m] = ((2 * l - 1) * z * P[l - 1][m] - (l + m - 1) * P[l - 2][m]) / (l - m);
  }
  // (x + i y)^m
  double re[8], im[8];
  re[0] = 1.0; im[0] = 0.0;
  for (int m = 1; m <= lmax; ++m) {
    re[m] = re[m - 1] * x - im[m - 1] * y;
    im[m] = re[m - 1] * y + im[m - 1] * x;
  }
  for (int l = 0; l <= lmax; ++l) {
    for (int m = 0; m <= l; ++m) {
      double r = 1.0;  // (l-m)!/(l+m)!
      for (int i = l - m + 1; i <= l + m; ++i) r /= i;
      double K = std::sqrt((2 * l + 1) / (4.0 * M_PI) * r);
      if (m == 0) {
        out[l * l + l] = K * P[l][0];
      } else {
        double c = std::sqrt(2.0) * K * P[l][m];
        out[l * l + l + m] = c * re[m];
        out[l * l + l - m] = c * im[m];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Dipole R_d (Eq. 4) for the PCA table.
// ---------------------------------------------------------------------------

double dipole_rd(double r, double sa, double ss, double eta) {
  const double st = sa + ss;
  const double alpha = ss / st;
  const double s = std::sqrt(3.0 * sa * st);
  const double zr = 1.0 / st;
  const double f = -1.440 / (eta * eta) + 0.710 / eta + 0.668 + 0.0636 * eta;
  const double A = (1.0 + f) / (1.0 - f);
  const double zv = zr * (1.0 + 4.0 * A / 3.0);
  const double dr = std::sqrt(r * r + zr * zr);
  const double dv = std::sqrt(r * r + zv * zv);
  const double tr = zr * (s + 1.0 / dr) * std::exp(-s * dr) / (dr * dr);
  const double tv = zv * (s + 1.0 / dv) * std::exp(-s * dv) / (dv * dv);
  return alpha / (4.0 * M_PI) * (tr + tv);
}

// One-sided (Hestenes) Jacobi SVD of A [m][n] (row-major, m >= n):
// returns singular values (descending) and right singular vectors as rows
// of Vt [n][n].
static void jacobi_svd(int m, int n, std::vector<double> A, std::vector<double> &sv,
                       std::vector<double> &Vt) {
  // Work on columns: store A column-major for contiguous column access.
  std::vector<double> C((size_t)m * n);
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) C[(size_t)j * m + i] = A[(size_t)i * n + j];
  std::vector<double> V((size_t)n * n, 0.0);  // column-major, V[:,j]
  for (int j = 0; j < n; ++j) V[(size_t)j * n + j] = 1.0;
  std::vector<double> nrm(n);
  for (int j = 0; j < n; ++j) {
    double s = 0;
    for (int i = 0; i < m; ++i) s += C[(size_t)j * m + i] * C[(size_t)j * m + i];
    nrm[j] = s;
  }
  for (int sweep = 0; sweep < 60; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n - 1; ++p) {
      for (int q = p + 1; q < n; ++q) {
        double *cp = &C[(size_t)p * m], *cq = &C[(size_t)q * m];
        double a = nrm[p], b = nrm[q], g = 0.0;
        for (int i = 0; i < m; ++i) g += cp[i] * cq[i];
        if (g == 0.0 || a == 0.0 || b == 0.0) continue;
        double rel = std::fabs(g) / (std::sqrt(a) * std::sqrt(b));
        if (!(rel > 1e-15)) continue;
        off = std::max(off, rel);
        double zeta = (b - a) / (2.0 * g);
        double t = (zeta >= 0 ? 1.0 : -1.0) / (std::fabs(zeta) + std::sqrt(1.0 + zeta * zeta));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = c * t;
        for (int i = 0; i < m; ++i) {
          double u = cp[i], w = cq[i];
          cp[i] = c * u - s * w;
          cq[i] = s * u + c * w;
        }
        double *vp = &V[(size_t)p * n], *vq = &V[(size_t)q * n];
        for (int i = 0; i < n; ++i) {
          double u = vp[i], w = vq[i];
          vp[i] = c * u - s * w;
          vq[i] = s * u + c * w;
        }
        double np_ = 0, nq_ = 0;
        for (int i = 0; i < m; ++i) { np_ += cp[i] * cp[i]; nq_ += cq[i] * cq[i]; }
        nrm[p] = np_;
        nrm[q] = nq_;
      }
    }
    if (off < 1e-15) break;
  }
  std::vector<int> order(n);
  for (int j = 0; j < n; ++j) order[j] = j;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return nrm[a] > nrm[b]; });
  sv.assign(n, 0.0);
  Vt.assign((size_t)n * n, 0.0);
  for (int r = 0; r < n; ++r) {
    int j = order[r];
    sv[r] = std::sqrt(nrm[j]);
    double *dst = &Vt[(size_t)r * n];
    const double *src = &V[(size_t)j * n];
    int imax = 0;
    for (int i = 0; i < n; ++i)
      if (std::fabs(src[i]) > std::fabs(src[imax])) imax = i;
    double sgn = src[imax] < 0 ? -1.0 : 1.0;
    for (int i = 0; i < n; ++i) dst[i] = sgn * src[i];
  }
}

}  // namespace tlt

using namespace tlt;

extern "C" tlt_status tlt_prepare_scene(tlt_scene *s) {
  if (!s) return fail(nullptr, TLT_E_ARG, "scene is NULL");
  const int N = s->n_vertices;
  if (N < 2 || s->n_faces < 1 || !s->vertices || !s->faces)
    return fail(nullptr, TLT_E_ARG, "need >= 2 vertices and >= 1 face");
  int lmax = (int)std::lround(std::sqrt((double)s->n_sh)) - 1;
  if (s->n_sh < 1 || (lmax + 1) * (lmax + 1) != s->n_sh || lmax > 7)
    return fail(nullptr, TLT_E_ARG, "n_sh must be (lmax+1)^2 with lmax <= 7");
  if (s->n_r < 2 || s->n_r > 1024) return fail(nullptr, TLT_E_ARG, "n_r must be in 2..1024");
  if (s->K < 1 || s->K > s->n_r) return fail(nullptr, TLT_E_ARG, "K must be in 1..n_r");
  if (!(s->r_max > 0.0) || !std::isfinite(s->r_max))
    return fail(nullptr, TLT_E_ARG, "r_max must be positive");
  for (int a = 0; a < 3; ++a) {
    if (s->mat_n[a] < 1 || !(s->mat_lo[a] > 0) || !(s->mat_hi[a] >= s->mat_lo[a]))
      return fail(nullptr, TLT_E_ARG, "bad material grid");
  }
  if (s->mat_lo[2] < 1.0) return fail(nullptr, TLT_E_ARG, "eta grid must be >= 1");
  if (!s->perm || !s->position || !s->area || !s->normal || !s->transfer || !s->r_nodes ||
      !s->basis)
    return fail(nullptr, TLT_E_ARG, "NULL output array");
  for (int f = 0; f < 3 * s->n_faces; ++f)
    if (s->faces[f] < 0 || s->faces[f] >= N) return fail(nullptr, TLT_E_ARG, "face index out of range");

  const double *V = s->vertices;
  // areas and normals in vertex order
  std::vector<double> area(N, 0.0), nrm(3 * (size_t)N, 0.0);
  for (int f = 0; f < s->n_faces; ++f) {
    const int32_t *t = &s->faces[3 * f];
    const double *a = &V[3 * t[0]], *b = &V[3 * t[1]], *c = &V[3 * t[2]];
    double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double x[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
    double ta = 0.5 * std::sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    for (int k = 0; k < 3; ++k) {
      area[t[k]] += ta / 3.0;
      for (int a2 = 0; a2 < 3; ++a2) nrm[3 * (size_t)t[k] + a2] += x[a2];
    }
  }
  morton_perm(N, V, s->perm);
  std::vector<double> y(s->n_sh);
  std::vector<double> ah(lmax + 1);
  for (int l = 0; l <= lmax; ++l) ah[l] = clamped_cosine_coeff(l);
  for (int p = 0; p < N; ++p) {
    const int v = s->perm[p];
    double n3[3] = {nrm[3 * (size_t)v], nrm[3 * (size_t)v + 1], nrm[3 * (size_t)v + 2]};
    double len = std::sqrt(n3[0] * n3[0] + n3[1] * n3[1] + n3[2] * n3[2]);
    if (!(len > 0.0) || !(area[v] > 0.0))
      return fail(nullptr, TLT_E_ARG, "degenerate vertex (zero area or normal)");
    for (int a = 0; a < 3; ++a) {
      n3[a] /= len;
      s->normal[3 * (size_t)p + a] = n3[a];
      s->position[3 * (size_t)p + a] = V[3 * (size_t)v + a];
    }
    s->area[p] = area[v];
    real_sh(lmax, n3, y.data());
    for (int l = 0; l <= lmax; ++l)
      for (int m = -l; m <= l; ++m)
        s->transfer[(size_t)p * s->n_sh + l * l + l + m] = ah[l] * y[l * l + l + m];
  }
  // r nodes and the PCA basis of the dipole table
  const int nr = s->n_r;
  for (int n = 0; n < nr; ++n) {
    double t = double(n) / double(nr - 1);
    s->r_nodes[n] = s->r_max * t * t;
  }
  std::vector<double> ga[3];
  for (int a = 0; a < 3; ++a) {
    ga[a].resize(s->mat_n[a]);
    for (int i = 0; i < s->mat_n[a]; ++i) {
      double t = s->mat_n[a] > 1 ? double(i) / (s->mat_n[a] - 1) : 0.0;
      if (a < 2) {
        ga[a][i] = std::exp(std::log(s->mat_lo[a]) + t * (std::log(s->mat_hi[a]) - std::log(s->mat_lo[a])));
      } else {
        ga[a][i] = s->mat_lo[a] + t * (s->mat_hi[a] - s->mat_lo[a]);
      }
    }
    ga[a].front() = s->mat_lo[a];
    if (s->mat_n[a] > 1) ga[a].back() = s->mat_hi[a];
  }
  const int nm = s->mat_n[0] * s->mat_n[1] * s->mat_n[2];
  const int rows = std::max(nm, nr);  // pad with zero rows so rows >= cols
  std::vector<double> M((size_t)rows * nr, 0.0);
  int row = 0;
  for (int i = 0; i < s->mat_n[0]; ++i)
    for (int j = 0; j < s->mat_n[1]; ++j)
      for (int k = 0; k < s->mat_n[2]; ++k, ++row)
        for (int n = 0; n < nr; ++n)
          M[(size_t)row * nr + n] = dipole_rd(s->r_nodes[n], ga[0][i], ga[1][j], ga[2][k]);
  std::vector<double> sv, Vt;
  jacobi_svd(rows, nr, M, sv, Vt);
  for (int k = 0; k < s->K; ++k)
    std::memcpy(&s->basis[(size_t)k * nr], &Vt[(size_t)k * nr], sizeof(double) * nr);
  if (s->singular_values) {
    int ns = std::min(nm, nr);
    for (int k = 0; k < ns; ++k) s->singular_values[k] = sv[k];
  }
  return TLT_OK;
}

// ---------------------------------------------------------------------------
// Transport rows (float64), precompute Step 1 of Sec. 3.2.
// ---------------------------------------------------------------------------

namespace tlt {

static inline int node_of(const double *rn, int nr, double r) {
  if (r >= rn[nr - 1]) return nr - 1;  // at or beyond the last node
  if (r <= 0.0) return 0;
  int n = (int)((nr - 1) * std::sqrt(r / rn[nr - 1]));
  if (n > nr - 2) n = nr - 2;
  if (n < 0) n = 0;
  while (n > 0 && r < rn[n]) --n;
  while (n < nr - 2 && r >= rn[n + 1]) ++n;
  return n;
}

static void haar_inplace(double *x, double *tmp, int64_t n) {
  const double h = 1.0 / std::sqrt(2.0);
  for (int64_t len = n; len > 1; len >>= 1) {
    const int64_t half = len >> 1;
    for (int64_t i = 0; i < half; ++i) {
      const double a = x[2 * i], b = x[2 * i + 1];
      tmp[i] = (a - b) * h;
      x[i] = (a + b) * h;
    }
    std::memcpy(x + half, tmp, sizeof(double) * half);
  }
}

static inline uint64_t mag_key(double v) {
  uint64_t u;
  std::memcpy(&u, &v, 8);
  return u & 0x7fffffffffffffffull;  // |v| as an ordered integer
}

// Keeps the n_keep entries of largest |x| (ties to the lower index);
// writes their indices ascending and their values.  The threshold is found
// from a histogram of the top 12 bits of |x| (ordered as integers), then an
// exact selection among the entries of the boundary bucket.
static void select_top(const double *x, int64_t n, int64_t n_keep, std::vector<uint64_t> &cand,
                       std::vector<uint32_t> &hist, int32_t *col, double *val) {
  if (n_keep >= n) {
    for (int64_t j = 0; j < n; ++j) { col[j] = (int32_t)j; val[j] = x[j]; }
    return;
  }
  hist.assign(4096, 0);
  for (int64_t j = 0; j < n; ++j) hist[mag_key(x[j]) >> 51]++;
  int64_t above = 0;
  int bucket = 4095;
  for (; bucket >= 0; --bucket) {
    if (above + hist[bucket] >= n_keep) break;
    above += hist[bucket];
  }
  cand.clear();
  for (int64_t j = 0; j < n; ++j) {
    const uint64_t k = mag_key(x[j]);
    if ((int)(k >> 51) == bucket) cand.push_back(k);
  }
  const int64_t need = n_keep - above;  // 1 <= need <= cand.size()
  std::nth_element(cand.begin(), cand.begin() + (cand.size() - need), cand.end());
  const uint64_t thr = cand[cand.size() - need];
  int64_t gt = above;
  for (uint64_t k : cand) gt += k > thr;
  int64_t ties = n_keep - gt, w = 0;
  for (int64_t j = 0; j < n; ++j) {
    const uint64_t k = mag_key(x[j]);
    bool take = k > thr;
    if (!take && k == thr && ties > 0) {
      take = true;
      --ties;
    }
    if (take) {
      col[w] = (int32_t)j;
      val[w] = x[j];
      ++w;
    }
  }
}

void host_build_rows(int n_rows, int n_cols, int K, int nr, int wavelet, int64_t n_keep,
                     const double *row_pos, const double *rn, const double *basis,
                     int32_t *col, double *val, int n_threads, int N, const double *pos) {
  // per-node slopes of every basis function, as in linear interpolation
  std::vector<double> slope((size_t)K * nr, 0.0);
  for (int k = 0; k < K; ++k)
    for (int m = 0; m + 1 < nr; ++m)
      slope[(size_t)k * nr + m] =
          (basis[(size_t)k * nr + m + 1] - basis[(size_t)k * nr + m]) / (rn[m + 1] - rn[m]);
  std::atomic<int64_t> next(0);
  const int64_t block = 16;
  auto worker = [&]() {
    std::vector<double> dr(N), x(n_cols), tmp(n_cols);
    std::vector<int32_t> node(N);
    std::vector<uint64_t> cand;
    std::vector<uint32_t> hist;
    for (;;) {
      const int64_t o0 = next.fetch_add(block);
      if (o0 >= n_rows) break;
      const int64_t o1 = std::min<int64_t>(n_rows, o0 + block);
      for (int64_t o = o0; o < o1; ++o) {
        const double *xo = &row_pos[3 * o];
        for (int i = 0; i < N; ++i) {
          const double dx = xo[0] - pos[3 * (size_t)i];
          const double dy = xo[1] - pos[3 * (size_t)i + 1];
          const double dz = xo[2] - pos[3 * (size_t)i + 2];
          const double r = std::sqrt(dx * dx + dy * dy + dz * dz);
          const int m = node_of(rn, nr, r);
          node[i] = m;
          dr[i] = r - rn[m];
        }
        for (int k = 0; k < K; ++k) {
          const double *bk = &basis[(size_t)k * nr];
          const double *sk = &slope[(size_t)k * nr];
          for (int i = 0; i < N; ++i) {
            const int m = node[i];
            x[i] = (m == nr - 1) ? bk[nr - 1] : sk[m] * dr[i] + bk[m];
          }
          for (int i = N; i < n_cols; ++i) x[i] = 0.0;
          if (wavelet == TLT_WAVELET_HAAR) haar_inplace(x.data(), tmp.data(), n_cols);
          const size_t rowoff = (size_t)(o * K + k) * (size_t)n_keep;
          select_top(x.data(), n_cols, n_keep, cand, hist, col + rowoff, val + rowoff);
        }
      }
    }
  };
  if (n_threads < 1) n_threads = 1;
  std::vector<std::thread> th;
  for (int t = 1; t < n_threads; ++t) th.emplace_back(worker);
  worker();
  for (auto &t : th) t.join();
}

}  // namespace tlt

extern "C" tlt_status tlt_build_rows(int32_t n_vertices, int32_t n_cols, int32_t K, int32_t n_r,
                                     int32_t wavelet, int64_t n_keep, const double *position,
                                     const double *r_nodes, const double *basis, int64_t n_rows,
                                     const int64_t *rows, int32_t *col_out, double *val_out) {
  const int N = n_vertices;
  if (N < 1 || K < 1 || n_r < 2 || n_rows < 0 || !position || !r_nodes || !basis ||
      (n_rows > 0 && (!rows || !col_out || !val_out)))
    return fail(nullptr, TLT_E_ARG, "bad arguments");
  if (wavelet != TLT_WAVELET_NONE && wavelet != TLT_WAVELET_HAAR)
    return fail(nullptr, TLT_E_ARG, "unknown wavelet");
  int64_t n_pad = 1;
  while (n_pad < N) n_pad <<= 1;
  if ((wavelet == TLT_WAVELET_HAAR && n_cols != n_pad) || (wavelet == TLT_WAVELET_NONE && n_cols != N))
    return fail(nullptr, TLT_E_ARG, "n_cols must be n_pad (Haar) or N (plain)");
  if (n_keep < 1 || n_keep > n_cols) return fail(nullptr, TLT_E_ARG, "n_keep out of range");
  std::vector<double> rp(3 * (size_t)n_rows);
  for (int64_t i = 0; i < n_rows; ++i) {
    if (rows[i] < 0 || rows[i] >= N) return fail(nullptr, TLT_E_ARG, "row out of range");
    for (int a = 0; a < 3; ++a) rp[3 * i + a] = position[3 * rows[i] + a];
  }
  unsigned h = std::thread::hardware_concurrency();
  host_build_rows((int)n_rows, n_cols, K, n_r, wavelet, n_keep, rp.data(), r_nodes, basis,
                  col_out, val_out, (int)std::max(1u, std::min(h, 16u)), N, position);
  return TLT_OK;
}
