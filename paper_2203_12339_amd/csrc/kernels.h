// Launch interface of the gfx950 kernels (internal to libtlt.so).
#pragma once
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace tlt {

// Storage tags for 16-bit values kept as raw bits in device memory.
struct bf16s { uint16_t u; };
struct f16s { uint16_t u; };

// Timing of the stage being profiled (thread-local, set by the host around
// the launches of one stage): the first launch of the stage writes `start`
// and every launch writes `stop`, as part of the kernel dispatch itself, so
// no marker packets sit between the kernels.
struct StageEvents {
  hipEvent_t start = nullptr, stop = nullptr;
  int launches = 0;
};
StageEvents &stage_events();

// Column mapping of a launch: column c = 3*q + ch of output set q uses
// lighting (n_light > 1 ? q : 0) and material (n_mat > 1 ? q : 0).
struct Cols {
  int C;        // 3 * n_out
  int n_out;
  int n_light;
  int n_mat;
};

// One launch for the material weights, the irradiance with its Haar
// transform, and the clearing of split output vertices; any part may be
// switched off by a zero block count.
struct PrepArgs {
  bool fp64;
  int tdt;                 // transfer storage (tlt.h codes)
  int Cs;                  // column stride of Ehat and gcol
  Cols cols;
  // material weights g_k
  int n_gk_blocks;         // n_mat * 3, or 0
  const double *theta;     // [n_mat][3][3]
  const double *rn;        // [nr]
  const double *basis;     // [K][nr]
  int nr, K;
  int gk_stage;            // stage the basis in LDS (K * nr small enough)
  double *g64, *dg64;      // [n_mat][3][K], [n_mat][3][K][3]
  void *gcol;              // [K][Cs] compute precision
  // material validation: flags [0] invalid, [1] outside the PCA table's
  // range, [2] an invalid (material, channel) index; host-visible memory
  int *mstat;
  int has_range;
  double mat_lo[3], mat_hi[3];
  // irradiance E = T L and its Haar transform
  int n_tl_blocks;         // n_chunks * Cs/16, or 0
  const void *T;           // [N][t_ld] storage tdt
  int N, n_sh, n_shp;
  int t_ld;                // row stride of T (0 = n_sh)
  int t_rows;              // rows of T (0 = N)
  const void *sh;          // [n_light][n_sh][3] compute precision; nullptr = identity
  const void *E;           // or: irradiance [n_light][N][3] (original order), replaces T L
  const int32_t *perm;     // Morton position -> original vertex id (with E)
  const void *area;        // [N] compute precision
  int haar, ch_rows, n_rows, n_chunks;
  void *ehat;              // [n_rows][Cs]
  void *partial;           // [n_chunks][Cs]
  void *ehat2;             // [n_rows][Cs] hi|lo 16-bit split of Ehat, or nullptr
  int split;               // 1 = bf16 hi/lo, 2 = f16 hi/lo
  // clearing of B at split vertices
  int n_zero_blocks;
  void *B;                 // [n_out][N][3]
  const int32_t *zero_v;   // original vertex ids
  int n_zero;
};
hipError_t launch_prep(const PrepArgs &a, hipStream_t st);
size_t prep_lds_bytes(const PrepArgs &a);

// Transport: streamed wavelet-sparse rows with K-term fusion.
struct StreamArgs {
  const int32_t *col;      // [N*K][n_keep]
  const void *val;         // [N*K][n_keep] storage
  int n_keep, K, N;
  const void *ehat;        // [n_rows][Cs]
  int Cs, C;
  const void *gcol;        // [K][Cs]
  const int32_t *perm;     // [N]
  void *B;                 // [n_out][N][3] or nullptr
  void *vsave;             // [N][K][vs_stride] or nullptr; row (perm[o], k)
  int vs_stride;
  int64_t R;               // N*K rows
  int n_waves;             // <= N
  int n_logical_blocks;    // set by launch_stream
  int epl;                 // entries per lane and step for 4-column tiles (0 = 8)
  int nt;                  // non-temporal loads of the transport
};
hipError_t launch_stream(StreamArgs a, int vdt, bool fp64, int cpl, hipStream_t st);
bool stream_cpl_supported(int cpl);
int stream_waves(int N, int K, int waves_per_cu);

// Transport on block-dense tiles (16-bit or f32 storage, f32 compute).
struct TileArgs {
  const int64_t *blk_off;  // [n_blocks+1] entry offsets (multiples of the k-step)
  const int32_t *ucol;     // entries' column ids
  const uint16_t *fmask;   // [entries / kstep] stored m-tiles per k-step
  const int64_t *foff;     // [n_blocks+1] fragment offsets
  const void *val;         // stored fragments (operand order)
  int V, K, R, n_blocks, N;
  const void *ehat;        // [n_rows][Cs] float32
  const void *ehat2;       // [n_rows][Cs] hi|lo split (16-bit kinds)
  int Cs, C;
  const void *gcol;        // [K][Cs] float32, or nullptr with B == nullptr
  const int32_t *perm;
  void *B;                 // [n_out][N][3] float32 or nullptr
  void *vsave;             // [N][K][vs_stride] or nullptr; row (perm[o], k)
  int vs_stride;
  int max_union;           // largest union of a block (entries)
  int shape;               // 16-bit kinds, 8 m-tiles: 100 MTW + 10 NT + IPT, 0 = built-in
  int stream_w;            // 1: the tile values exceed the Infinity Cache (W streams once)
  int sparse;              // 1: fragment-sparse blocks (rows (k, o), step masks)
  int wn, kc, n_groups, uc_offset, mk_offset;  // set by launch_tiles
};
hipError_t launch_tiles(const TileArgs &a, int vdt, hipStream_t st);
int tile_kstep(int vdt);
// Largest block (rows V*K) the tile kernel takes for a storage type.
int tile_max_rows(int vdt);

// Outgoing Fresnel factor (1/pi) F_t(eta, w_o) applied to B in place.
hipError_t launch_view(void *B, const void *cosv, const double *theta, Cols cols, int N,
                       const int32_t *perm, bool fp64, hipStream_t st);

// Material-only update: B from kept v_k [N][K][Cs] (vertices in original
// order) and gcol.
hipError_t launch_combine(const void *V, int Cs, const void *gcol, int K, int N, int C, void *B,
                          bool fp64, hipStream_t st);

// Folded lighting transport: B = sum_k g_k P_k L (P_k = W_k H (A o T), stored
// [N][K][Psh], vertices in original order).
// With P16 (float32 compute only) the product runs on the FP16 copy of P
// written by launch_fold_pack, whose scale 1/sp is p16_inv.
hipError_t launch_folded(const void *P, int Psh, int n_sh, int K, const void *gcol, int Cs,
                         const void *sh, Cols cols, int N, void *B, bool fp64, void *scratch,
                         hipStream_t st, const void *P16 = nullptr, float p16_inv = 0.f);
size_t folded_scratch_bytes(int K, int Psh, int Cs, bool fp64);
// FP16 copy of P for the folded product: J = K Psh contraction indices in
// S = ceil(J / 32) steps of 32, one 1 KB A-operand fragment per (16-row
// tile, step); largest J it takes (0 if none).
constexpr int FOLD16_MAX_STEPS = 16;
size_t fold16_bytes(int N, int J);
// largest |P| (float bits) into *absmax (a device word the caller zeroed)
hipError_t launch_fold_absmax(const float *P, int64_t n, unsigned *absmax, hipStream_t st);
// P16 = sp * P in fragment order (sp a power of two)
hipError_t launch_fold_pack(const float *P, int N, int J, float sp, void *P16, hipStream_t st);

// Adjoint from Z_k = P_k^T dB: partial rows, then the final reduction.
// `partial` holds adjoint_partial_bytes(N, K, n_sh, C, fp64) bytes.
hipError_t launch_adjoint(const void *dB, const void *P, int Psh, const void *gcol, int Cs,
                          const void *sh, const double *dg64, int N, int K, int n_sh, Cols cols,
                          bool fp64, void *partial, size_t partial_bytes, void *dSH, double *dTheta,
                          hipStream_t st);
size_t adjoint_partial_bytes(int N, int K, int n_sh, int C, bool fp64);

// Load-time transport build on the device: kernel rows, Haar transform and
// exact top-n selection for vertices [o0, o0 + nv) and the k of one group.
struct BuildArgs {
  const double *pos;       // [N][3] Morton order
  const double *rn;        // [nr]
  const double *basis;     // [K][nr]
  const double *slope;     // [K][nr] (b[m+1] - b[m]) / (r[m+1] - r[m])
  int N, n_cols, K, nr, haar;
  double hsq;              // 1/sqrt(2) as the host computes it
  int64_t n_keep;
  int o0, nv, kg0;
  int all;                 // n_keep == n_cols: every coefficient, in order
  int max_chunks;          // LDS rows of chunk sums
  int32_t *scol;           // [nv*K][n_keep] unsorted kept columns
  double *sval;            // [nv*K][n_keep]
  int32_t *col;            // final rows [N*K][n_keep]
  void *val;               // storage type vdt
  int vdt;
  int *status;             // nonzero after a failed internal check
  // BF16 storage: for columns j < head_cols, the BF16 rounding of the
  // residual W - bf16(W) at [global row][j] (zero-initialised), or nullptr
  uint16_t *res;
  int head_cols;
};
size_t build_select_lds(int KG, int nr, int max_chunks);
int build_chunk_columns();
int build_max_group();
int build_sort_max();
hipError_t launch_build_select(const BuildArgs &a, int KG, hipStream_t st);
hipError_t launch_build_sort(const BuildArgs &a, hipStream_t st);

// Fragment-sparse (`order`) or dense tiles from the device rows (count
// pass, then fill pass).  A block holds V consecutive Morton vertices, i.e.
// R = V*K rows, ordered (k, o) (row k*V + o - v0) when sparse, else (o, k).  Its entries are the union U of the kept
// columns of those rows (with residuals, BF16 storage and `res` non-null,
// the union's h columns below head_cols once more, whose values are the
// BF16 residuals of those rows' entries, so the product adds W - bf16(W)
// for the coarsest columns).  With `order`, the entries are sorted by the
// first and last 16-row m-tile that keeps them (then by entry), which
// gathers the entries kept by the same rows into the same k-steps; padded
// to a multiple of `kstep` (padding entries read column 0 with zero
// weights).  Per k-step s a mask of the m-tiles t with a kept entry in it;
// only those (s, t) fragments are stored, in (s, t) order, each as the
// matrix-instruction operand: lane l, element i < kpl = kstep/4 holds
// W[row 16t + l%16][entry s*kstep + kpl*(l/16) + i].  Without `order` (or
// for unions above 8192 entries) the entries stay in column order and every
// fragment is stored (the mask of every step is full).
struct TileBuildArgs {
  const int32_t *col;      // [N*K][n_keep] ascending
  const void *val;         // storage values (esz bytes)
  int esz;
  int N, K, V;
  int64_t n_keep;
  int n_words;             // ceil(n_cols / 32)
  int n_blocks, kstep;
  bool order;              // sort the entries by m-tile pattern (fits the LDS)
  int64_t *count;          // count pass: padded entries per block
  int64_t *fcount;         // count pass: stored fragments per block
  const int64_t *blk_off;  // fill pass: [n_blocks+1] entry offsets
  const int64_t *frag_off; // fill pass: [n_blocks+1] fragment offsets
  int32_t *ucol;           // [entries]
  uint16_t *mask;          // [entries / kstep] m-tile mask per k-step
  void *tval;              // [fragments][64][kpl] storage values, zero-initialised
  const uint16_t *res;     // [N*K][head_cols] residuals, or nullptr
  int head_cols;           // <= 64
};
size_t tile_build_lds(int n_words, bool order);
hipError_t launch_tile_count(const TileBuildArgs &a, hipStream_t st);
hipError_t launch_tile_fill(const TileBuildArgs &a, hipStream_t st);

// Read-bandwidth probe: streams `bytes` of buf; out [blocks * 4].
hipError_t launch_read_probe(const void *buf, int64_t bytes, uint32_t *out, int blocks, hipStream_t st);

// Storage conversion of float64 values to device storage type.
hipError_t launch_quantize(const double *src, void *dst, int vdt, int64_t n, hipStream_t st);
// The same for entries e0 .. e0+n of caller-given rows (col: all columns on
// the device), writing the BF16 residual words of the columns below
// head_cols into res [rows][head_cols] when res is not null.
hipError_t launch_quantize_rows(const double *src, const int32_t *col, void *val, int vdt, int64_t e0,
                                int64_t n, int64_t n_keep, uint16_t *res, int head_cols, hipStream_t st);

}  // namespace tlt
