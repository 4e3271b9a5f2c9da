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

namespace tlt {

// Block-dense transport tiles.  A block holds V consecutive Morton vertices,
// i.e. R = V*K rows (o, k).  Its columns are the sorted union U of the kept
// columns of those rows, padded to a multiple of `kstep` (padding columns
// point at column 0 with zero weights).  Values are stored densely over
// [U x R] in MFMA fragment order: for k-step s, m-tile t (16 rows), lane l
// and element i < kpl the value W[row = 16t + l%16][u = s*kstep + kpl*(l/16)
// + i], where kpl = kstep/4.
struct TileBuild {
  int V = 16, K = 0, kstep = 4;
  int64_t n_blocks = 0;
  std::vector<int64_t> blk_off;   // [n_blocks+1] offsets in union entries
  std::vector<int32_t> ucol;      // [total union entries]
  std::vector<uint16_t> v16;      // values when stored as 16-bit
  std::vector<float> v32;         // values when stored as float32
};

// Appends the tiles of `nv` vertices (a multiple of V unless it is the last
// chunk) whose ELL rows are col/val [nv][K][n_keep] (float64 values).
// vdt selects the stored value type (tlt.h codes F32/BF16/F16).
void tiles_append(TileBuild &tb, int nv, int n_cols, int64_t n_keep, const int32_t *col,
                  const double *val, int vdt, int n_threads);

uint16_t f32_to_bf16(float f);
uint16_t f32_to_f16(float f);

}  // namespace tlt
