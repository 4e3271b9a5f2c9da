// Internal declarations shared by the host precompute and the device API.
#pragma once
#include <cstdint>
#include <string>

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

}  // namespace tlt
