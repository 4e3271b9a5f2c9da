// Internal declarations shared by the host precompute and the device API.
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tlt.h"

namespace tlt {

extern thread_local std::string g_thread_error;

// Records msg in *dst (if not NULL) and in the calling thread's error slot.
tlt_status fail(std::string *dst, tlt_status st, const std::string &msg);

// Dipole diffuse reflectance of Eq. (4), float64.
double dipole_rd(double r, double sa, double ss, double eta);

// Transport rows in float64 (precompute Step 1, Sec. 3.2): for each of the
// n_rows output points row_pos[o] and term k, row o*K+k of col/val receives
// the n_keep kept (column, value) pairs, columns ascending.  pos holds all N
// Morton-ordered vertices [N][3]; n_cols = n_pad (Haar) or N (plain).
// Uses n_threads host threads.
void host_build_rows(int n_rows, int n_cols, int K, int nr, int wavelet, int64_t n_keep,
                     const double *row_pos, const double *rn, const double *basis,
                     int32_t *col, double *val, int n_threads, int N, const double *pos);

// Spatial compression of the Step-1 rows (precompute Step 2 of Sec. 3.2):
// CSR over the output coefficient u of the kept entries of Z_k = w_1 W_k^S,
// column word (k << 24) | j, entries of a row in (k, j) order.
struct SpatialCsr {
  std::vector<int64_t> rowptr;     // [N + 1]
  std::vector<uint32_t> col;       // [nnz]
  std::vector<double> val;         // [nnz]
  std::vector<int> sizes;          // list length split at each level, finest first
  std::vector<int64_t> nnz_k;      // kept entries per term
  std::vector<double> energy_kept; // retained energy fraction per term
};

// Lengths split by the CDF 9/7 levels of a list of n (finest first);
// levels = 0 splits while at least 8 entries remain.
std::vector<int> cdf97_sizes(int n, int levels);

// w_1^{-1} as a sparse matrix (CSR over the output position o: the
// coefficients u and weights with (w_1^{-1} y)[o] = sum w y[u]), from the
// synthesis of every unit coefficient (Step 5 of Sec. 4).
void synthesis_build(int N, const std::vector<int> &sizes, int n_threads, std::vector<int32_t> &rowptr,
                     std::vector<int32_t> &col, std::vector<double> &w);

// col/val: [N][K][n_keep] float64 Step-1 rows (Morton row order).  energy in
// (0, 1]; levels as in cdf97_sizes.  Runs on n_threads host threads.
tlt_status spatial_build(int N, int n_cols, int K, int64_t n_keep, const int32_t *col,
                         const double *val, double energy, int levels, int n_threads,
                         SpatialCsr &out, std::string *err);

}  // namespace tlt
