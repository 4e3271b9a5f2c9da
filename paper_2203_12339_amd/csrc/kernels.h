// Launch interface of the gfx950 kernels (internal to libtlt.so).
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>

namespace tlt {

// Storage tags for 16-bit values kept as raw bits in device memory.
struct bf16s { uint16_t u; };
struct f16s { uint16_t u; };

// Column mapping of a launch: column c = 3*q + ch of output set q.
struct Cols {
  int C;        // 3 * n_out
  int n_out;
  int n_light;
  int n_mat;
};

// a1: g[m][ch][k], dg[m][ch][k][p] in float64 and the per-column weights
// gcol[k][Cs] (compute precision, zero for padded columns).
hipError_t launch_gk(const double *theta, const double *rn, const double *basis, int nr, int K,
                     double *g64, double *dg64, void *gcol, bool fp64, int Cs, Cols cols,
                     hipStream_t st);

// Lighting matrix Lm[lm][Cs] (compute precision) from sh [n_light][n_sh][3];
// identity (Lm[lm][lm] = 1) when sh == nullptr.  Rows up to n_shp.
hipError_t launch_lmat(const void *sh, bool fp64, int n_sh, int n_shp, int Cs, Cols cols,
                       void *Lm, hipStream_t st);

// a2 + a3: Ehat = Haar(pad(A o (T Lm))) over rows (wavelet) or A o (T Lm).
// T [N][n_sh] storage tdt; area [N] (compute precision); ehat [n_rows][Cs];
// partial [n_chunks][Cs] scratch for the coarse levels.
hipError_t launch_tl_haar(const void *T, int tdt, int N, int n_sh, int n_shp, const void *Lm,
                          const void *area, bool fp64, bool haar, int n_rows, int Cs,
                          void *ehat, void *partial, hipStream_t st);

// a4 + a5: B[q][perm[o]][ch] = sum_k gcol[k][c] sum_j W[o*K+k][j] ehat[j][c]
// and optionally vsave[k][o][vs_stride] = per-k sums. B may be null.
hipError_t launch_transport(const int32_t *col, const void *val, int vdt, int64_t n_keep, int K,
                            int N, const void *ehat, int Cs, int C, int cpl, const void *gcol,
                            const int32_t *perm, void *B, void *vsave, int vs_stride, bool fp64,
                            hipStream_t st);
bool transport_cpl_supported(int cpl, bool fp64);

// Material-only update: B from saved v_k [K][N][Cs] and gcol.
hipError_t launch_combine(const void *V, int Cs, const void *gcol, int K, int N, int C,
                          const int32_t *perm, void *B, bool fp64, hipStream_t st);

// a6: partial sums over vertex blocks, then the final reduction.
hipError_t launch_adjoint(const void *dB, const void *V, int Cs, const void *P, int Psh,
                          const void *gcol, const double *dg64, const int32_t *perm, int N, int K,
                          int n_sh, Cols cols, bool fp64, void *partial, size_t partial_bytes,
                          void *dSH, double *dTheta, hipStream_t st);
size_t adjoint_partial_bytes(int N, int K, int n_sh, int C, bool fp64);

// Storage conversion of float64 host values to device storage type.
hipError_t launch_quantize(const double *src, void *dst, int vdt, int64_t n, hipStream_t st);

}  // namespace tlt
