// gfx950 kernels of the translucent-transport library.
//
//   k_gk         a1  material weights g_k (Sec. 2.2, Step 3 of Sec. 4), float64
//   k_lmat       lighting matrix for the transfer product
//   k_tl_haar    a2+a3 E = T L (MFMA), area weight, Haar levels inside a chunk
//   k_haar_top   a3  the coarse Haar levels over the chunk sums (Eq. 8)
//   k_transport  a4+a5 wavelet-sparse transport with K-term fusion (Eq. 7,
//                Steps 2 and 4 of Sec. 4), store in original vertex order
//   k_adj_*      a6  adjoint reductions (lighting and material gradients)
//   k_quantize   storage conversion at load time
//
// Wave size 64 everywhere.  All reductions run in a fixed order, so results
// are deterministic run to run.

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.h"

namespace tlt {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------------------
// Storage loads (every storage type widens exactly to the compute type).
// ---------------------------------------------------------------------------

template <typename VT, typename CT> __device__ __forceinline__ CT ld(const VT *p, int64_t i);
template <> __device__ __forceinline__ double ld<double, double>(const double *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ float ld<float, float>(const float *p, int64_t i) { return p[i]; }
template <> __device__ __forceinline__ double ld<float, double>(const float *p, int64_t i) { return (double)p[i]; }
template <> __device__ __forceinline__ float ld<bf16s, float>(const bf16s *p, int64_t i) {
  return __uint_as_float(((uint32_t)p[i].u) << 16);
}
template <> __device__ __forceinline__ float ld<f16s, float>(const f16s *p, int64_t i) {
  return (float)__builtin_bit_cast(_Float16, p[i].u);
}

template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
  return v;
}

// ---------------------------------------------------------------------------
// a1: dipole R_d (Eq. 4) and its parameter derivatives, projected on b_k.
// ---------------------------------------------------------------------------

struct RdGrad {
  double R, da, ds, de;
};

__device__ inline void pole(double z, double d, double s, double &f, double &fs, double &fz) {
  const double e = exp(-s * d);
  const double id = 1.0 / d;
  const double h = (s + id) * e * id * id;
  f = z * h;
  fs = -s * z * e * id;  // partial w.r.t. sigma_tr
  const double hp = -e * id * id * (s * s + 3.0 * s * id + 3.0 * id * id);
  fz = h + z * hp * (z * id);  // total w.r.t. z through d = sqrt(r^2 + z^2)
}

__device__ inline RdGrad rd_grad(double r, double sa, double ss, double eta) {
  const double st = sa + ss;
  const double alpha = ss / st;
  const double s = sqrt(3.0 * sa * st);
  const double zr = 1.0 / st;
  const double f = -1.440 / (eta * eta) + 0.710 / eta + 0.668 + 0.0636 * eta;
  const double A = (1.0 + f) / (1.0 - f);
  const double cv = 1.0 + 4.0 * A / 3.0;
  const double zv = zr * cv;
  const double dr = sqrt(r * r + zr * zr);
  const double dv = sqrt(r * r + zv * zv);
  double fr, frs, frz, fv, fvs, fvz;
  pole(zr, dr, s, fr, frs, frz);
  pole(zv, dv, s, fv, fvs, fvz);
  const double S = fr + fv;
  const double k4 = 1.0 / (4.0 * M_PI);
  // d(sigma_tr), d(alpha'), d(z_r) per parameter; z_v = cv z_r.
  const double dfd = 2.880 / (eta * eta * eta) - 0.710 / (eta * eta) + 0.0636;
  const double dA = 2.0 / ((1.0 - f) * (1.0 - f)) * dfd;
  const double dzr = -1.0 / (st * st);
  RdGrad g;
  g.R = alpha * k4 * S;
  {
    const double dal = -ss / (st * st), dsg = 3.0 * (st + sa) / (2.0 * s);
    g.da = dal * k4 * S + alpha * k4 * ((frs + fvs) * dsg + frz * dzr + fvz * cv * dzr);
  }
  {
    const double dal = sa / (st * st), dsg = 3.0 * sa / (2.0 * s);
    g.ds = dal * k4 * S + alpha * k4 * ((frs + fvs) * dsg + frz * dzr + fvz * cv * dzr);
  }
  g.de = alpha * k4 * fvz * (zr * 4.0 / 3.0 * dA);
  return g;
}

// grid: n_mat*3 workgroups of 256 threads.
__global__ __launch_bounds__(256) void k_gk(const double *__restrict__ theta,
                                            const double *__restrict__ rn,
                                            const double *__restrict__ basis, int nr, int K,
                                            double *__restrict__ g64, double *__restrict__ dg64,
                                            void *__restrict__ gcol, int fp64, int Cs, Cols cols) {
  extern __shared__ double sh_q[];  // [4][nr]
  const int mc = blockIdx.x;        // m*3 + ch
  const int m = mc / 3, ch = mc % 3;
  const double sa = theta[mc * 3 + 0], ss = theta[mc * 3 + 1], eta = theta[mc * 3 + 2];
  for (int n = threadIdx.x; n < nr; n += blockDim.x) {
    RdGrad g = rd_grad(rn[n], sa, ss, eta);
    sh_q[n] = g.R;
    sh_q[nr + n] = g.da;
    sh_q[2 * nr + n] = g.ds;
    sh_q[3 * nr + n] = g.de;
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 4 * K; t += blockDim.x) {
    const int k = t / 4, qn = t % 4;
    const double *b = basis + (size_t)k * nr;
    const double *q = sh_q + (size_t)qn * nr;
    double acc = 0.0;
    for (int n = 0; n < nr; ++n) acc = fma(q[n], b[n], acc);
    if (qn == 0) {
      g64[(size_t)mc * K + k] = acc;
      for (int o = 0; o < cols.n_out; ++o) {
        const int mo = cols.n_mat > 1 ? o : 0;
        if (mo != m) continue;
        const int c = 3 * o + ch;
        if (fp64)
          ((double *)gcol)[(size_t)k * Cs + c] = acc;
        else
          ((float *)gcol)[(size_t)k * Cs + c] = (float)acc;
      }
    } else {
      dg64[((size_t)mc * K + k) * 3 + (qn - 1)] = acc;
    }
  }
}

hipError_t launch_gk(const double *theta, const double *rn, const double *basis, int nr, int K,
                     double *g64, double *dg64, void *gcol, bool fp64, int Cs, Cols cols,
                     hipStream_t st) {
  size_t lds = sizeof(double) * 4 * nr;
  hipLaunchKernelGGL(k_gk, dim3(cols.n_mat * 3), dim3(256), lds, st, theta, rn, basis, nr, K,
                     g64, dg64, gcol, (int)fp64, Cs, cols);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Lighting matrix.
// ---------------------------------------------------------------------------

template <typename CT>
__global__ void k_lmat(const CT *__restrict__ sh, int n_sh, int n_shp, int Cs, Cols cols,
                       CT *__restrict__ Lm) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_shp * Cs) return;
  const int lm = i / Cs, c = i % Cs;
  CT v = 0;
  if (lm < n_sh) {
    if (sh == nullptr) {
      v = (c == lm) ? CT(1) : CT(0);
    } else if (c < cols.C) {
      const int q = c / 3, ch = c % 3;
      const int l = cols.n_light > 1 ? q : 0;
      v = sh[((size_t)l * n_sh + lm) * 3 + ch];
    }
  }
  Lm[i] = v;
}

hipError_t launch_lmat(const void *sh, bool fp64, int n_sh, int n_shp, int Cs, Cols cols,
                       void *Lm, hipStream_t st) {
  const int n = n_shp * Cs;
  const int blocks = (n + 255) / 256;
  if (fp64)
    hipLaunchKernelGGL(k_lmat<double>, dim3(blocks), dim3(256), 0, st, (const double *)sh, n_sh,
                       n_shp, Cs, cols, (double *)Lm);
  else
    hipLaunchKernelGGL(k_lmat<float>, dim3(blocks), dim3(256), 0, st, (const float *)sh, n_sh,
                       n_shp, Cs, cols, (float *)Lm);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a2 + a3: E = T Lm on MFMA, times area, then the Haar levels that stay
// inside a chunk of CH rows.  grid (n_chunks, Cs/16), 256 threads: wave w
// owns rows [64w, 64w+64) of the chunk as four 16x16 MFMA tiles.
//
// MFMA 16x16x4 operand layout (f32 and f64 alike): lane l supplies
// A[l%16][l/16] and B[l/16][l%16].  Result element v of lane l is
// D[4*(l/16)+v][l%16] for f32 but D[(l/16)+4v][l%16] for f64 (checked
// on gfx950 with a probe of known operands).
// ---------------------------------------------------------------------------

constexpr int TL_CH = 256;  // rows per chunk (power of two)
constexpr int TL_LDS_STRIDE = 17;

__device__ __forceinline__ f32x4 mfma16(float a, float b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f64x4 mfma16(double a, double b, f64x4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

template <typename CT> struct vec4_of;
template <> struct vec4_of<float> {
  typedef f32x4 type;
  static __device__ __forceinline__ int row(int lk, int v) { return 4 * lk + v; }
};
template <> struct vec4_of<double> {
  typedef f64x4 type;
  static __device__ __forceinline__ int row(int lk, int v) { return lk + 4 * v; }
};

template <typename TT, typename CT>
__global__ __launch_bounds__(256) void k_tl_haar(const TT *__restrict__ T, int N, int n_sh,
                                                 int n_shp, const CT *__restrict__ Lm,
                                                 const CT *__restrict__ area, int haar, int ch_rows,
                                                 int n_rows, int Cs, CT *__restrict__ ehat,
                                                 CT *__restrict__ partial) {
  typedef typename vec4_of<CT>::type V4;
  __shared__ CT x[TL_CH * TL_LDS_STRIDE];
  const int chunk = blockIdx.x;
  const int c0 = blockIdx.y * 16;
  const int i0 = chunk * ch_rows;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;

  // E tile via MFMA: rows i0 + 64*wave + 16*t + (..), columns c0..c0+15.
  if (64 * wave < ch_rows) {
    V4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = V4{0, 0, 0, 0};
    for (int kk = 0; kk < n_shp; kk += 4) {
      const int kcol = kk + lk;
      const CT b = Lm[(size_t)kcol * Cs + c0 + li];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int r = i0 + 64 * wave + 16 * t + li;
        CT a = 0;
        if (r < N && kcol < n_sh && 64 * wave + 16 * t < ch_rows) a = ld<TT, CT>(T, (int64_t)r * n_sh + kcol);
        acc[t] = mfma16(a, b, acc[t]);
      }
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = 64 * wave + 16 * t + vec4_of<CT>::row(lk, v);  // local row
        const int r = i0 + lr;
        const CT ar = (r < N) ? area[r] : CT(0);
        if (lr < ch_rows) x[lr * TL_LDS_STRIDE + li] = acc[t][v] * ar;
      }
    }
  }
  __syncthreads();

  if (!haar) {
    for (int idx = threadIdx.x; idx < ch_rows * 16; idx += 256) {
      const int lr = idx >> 4, c = idx & 15;
      const int r = i0 + lr;
      if (r < n_rows) ehat[(size_t)r * Cs + c0 + c] = x[lr * TL_LDS_STRIDE + c];
    }
    return;
  }

  // Haar levels inside the chunk.  At each step the chunk holds `len`
  // scaling values; pair i produces detail index (len/2)*(n_chunks+chunk)+i.
  const CT h = CT(0.70710678118654752440);
  const int n_chunks = n_rows / ch_rows;
  for (int len = ch_rows; len > 1; len >>= 1) {
    const int half = len >> 1;
    CT sv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = threadIdx.x + 256 * u;
      if (idx < half * 16) {
        const int i = idx >> 4, c = idx & 15;
        const CT a = x[(2 * i) * TL_LDS_STRIDE + c];
        const CT b = x[(2 * i + 1) * TL_LDS_STRIDE + c];
        const int64_t j = (int64_t)half * (n_chunks + chunk) + i;
        ehat[j * Cs + c0 + c] = (a - b) * h;
        sv[u] = (a + b) * h;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = threadIdx.x + 256 * u;
      if (idx < half * 16) x[(idx >> 4) * TL_LDS_STRIDE + (idx & 15)] = sv[u];
    }
    __syncthreads();
  }
  if (threadIdx.x < 16) {
    const CT s = x[threadIdx.x];
    if (n_chunks == 1)
      ehat[c0 + threadIdx.x] = s;
    else
      partial[(size_t)chunk * Cs + c0 + threadIdx.x] = s;
  }
}

// Coarse Haar levels over the n_chunks chunk sums of one column.
// grid: Cs workgroups of 256 threads; LDS holds n_chunks values.
template <typename CT>
__global__ __launch_bounds__(256) void k_haar_top(const CT *__restrict__ partial, int n_chunks,
                                                  int Cs, CT *__restrict__ ehat) {
  extern __shared__ unsigned char raw[];
  CT *s = reinterpret_cast<CT *>(raw);
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < n_chunks; i += 256) s[i] = partial[(size_t)i * Cs + c];
  __syncthreads();
  const CT h = CT(0.70710678118654752440);
  for (int len = n_chunks; len > 1; len >>= 1) {
    const int half = len >> 1;
    CT sv[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = threadIdx.x + 256 * u;
      if (i < half) {
        const CT a = s[2 * i], b = s[2 * i + 1];
        ehat[(size_t)(half + i) * Cs + c] = (a - b) * h;
        sv[u] = (a + b) * h;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = threadIdx.x + 256 * u;
      if (i < half) s[i] = sv[u];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) ehat[c] = s[0];
}

template <typename TT, typename CT>
static void tl_haar_launch(const void *T, int N, int n_sh, int n_shp, const void *Lm,
                           const void *area, bool haar, int n_rows, int Cs, void *ehat,
                           void *partial, hipStream_t st) {
  const int ch_rows = n_rows < TL_CH ? n_rows : TL_CH;
  const int n_chunks = (n_rows + ch_rows - 1) / ch_rows;
  hipLaunchKernelGGL((k_tl_haar<TT, CT>), dim3(n_chunks, Cs / 16), dim3(256), 0, st,
                     (const TT *)T, N, n_sh, n_shp, (const CT *)Lm, (const CT *)area, (int)haar,
                     ch_rows, n_rows, Cs, (CT *)ehat, (CT *)partial);
  if (haar && n_chunks > 1) {
    hipLaunchKernelGGL((k_haar_top<CT>), dim3(Cs), dim3(256), sizeof(CT) * n_chunks, st,
                       (const CT *)partial, n_chunks, Cs, (CT *)ehat);
  }
}

hipError_t launch_tl_haar(const void *T, int tdt, int N, int n_sh, int n_shp, const void *Lm,
                          const void *area, bool fp64, bool haar, int n_rows, int Cs,
                          void *ehat, void *partial, hipStream_t st) {
  // 0 = f64, 1 = f32, 2 = bf16, 3 = f16 (tlt.h storage codes)
  if (fp64) {
    if (tdt == 0)
      tl_haar_launch<double, double>(T, N, n_sh, n_shp, Lm, area, haar, n_rows, Cs, ehat, partial, st);
    else
      return hipErrorInvalidValue;
  } else {
    switch (tdt) {
      case 1: tl_haar_launch<float, float>(T, N, n_sh, n_shp, Lm, area, haar, n_rows, Cs, ehat, partial, st); break;
      case 2: tl_haar_launch<bf16s, float>(T, N, n_sh, n_shp, Lm, area, haar, n_rows, Cs, ehat, partial, st); break;
      case 3: tl_haar_launch<f16s, float>(T, N, n_sh, n_shp, Lm, area, haar, n_rows, Cs, ehat, partial, st); break;
      default: return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a4 + a5: wavelet-sparse transport with K-term fusion.
//
// One wave per output vertex o (Morton position).  Lanes split the n_keep
// entries of each row (o, k); every lane gathers the CPL consecutive
// columns [c0, c0+CPL) of Ehat row j for its entries and accumulates in
// registers; at the end of row k the lane folds g_k[c] into its running
// radiance.  One butterfly reduction per vertex (and per row when v_k is
// saved).  Workgroups are remapped so that each XCD receives a contiguous
// range of vertices (Morton-adjacent vertices share Ehat rows in its L2).
// ---------------------------------------------------------------------------

template <typename CT, int CPL> struct RowLoad;
template <int CPL> struct RowLoad<float, CPL> {
  static __device__ __forceinline__ void load(const float *p, float (&v)[CPL]) {
    static_assert(CPL % 4 == 0, "float rows load as float4");
#pragma unroll
    for (int q = 0; q < CPL / 4; ++q) {
      const float4 t = reinterpret_cast<const float4 *>(p)[q];
      v[4 * q] = t.x; v[4 * q + 1] = t.y; v[4 * q + 2] = t.z; v[4 * q + 3] = t.w;
    }
  }
};
template <int CPL> struct RowLoad<double, CPL> {
  static __device__ __forceinline__ void load(const double *p, double (&v)[CPL]) {
    static_assert(CPL % 2 == 0, "double rows load as double2");
#pragma unroll
    for (int q = 0; q < CPL / 2; ++q) {
      const double2 t = reinterpret_cast<const double2 *>(p)[q];
      v[2 * q] = t.x; v[2 * q + 1] = t.y;
    }
  }
};

template <typename VT, typename CT, int CPL, int U>
__global__ __launch_bounds__(256) void k_transport(
    const int32_t *__restrict__ col, const VT *__restrict__ val, int64_t n_keep, int K, int N,
    const CT *__restrict__ ehat, int Cs, int C, const CT *__restrict__ gcol,
    const int32_t *__restrict__ perm, CT *__restrict__ B, CT *__restrict__ vsave, int vs_stride,
    int n_logical_blocks) {
  // XCD-aware remap: hardware block b runs on XCD b % 8.
  const int per = (n_logical_blocks + 7) >> 3;
  const int lb = (blockIdx.x & 7) * per + (blockIdx.x >> 3);
  if (lb >= n_logical_blocks) return;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int o = lb * 4 + wave;
  if (o >= N) return;
  const int c0 = blockIdx.y * CPL;

  CT bacc[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) bacc[c] = 0;

  for (int k = 0; k < K; ++k) {
    const int64_t base = ((int64_t)o * K + k) * n_keep;
    CT acc[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) acc[c] = 0;
    for (int64_t e = lane; e < n_keep; e += 64 * U) {
      int jj[U];
      CT ww[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t idx = e + 64 * u;
        if (idx < n_keep) {
          jj[u] = col[base + idx];
          ww[u] = ld<VT, CT>(val, base + idx);
        } else {
          jj[u] = 0;
          ww[u] = 0;
        }
      }
      CT ev[U][CPL];
#pragma unroll
      for (int u = 0; u < U; ++u) RowLoad<CT, CPL>::load(ehat + (int64_t)jj[u] * Cs + c0, ev[u]);
#pragma unroll
      for (int u = 0; u < U; ++u)
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = fma(ww[u], ev[u][c], acc[c]);
    }
    const CT *gk = gcol + (size_t)k * Cs + c0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) bacc[c] = fma(gk[c], acc[c], bacc[c]);
    if (vsave != nullptr) {
      CT mine = 0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) {
        const CT t = wave_sum(acc[c]);
        if (lane == c) mine = t;
      }
      if (lane < CPL) vsave[((int64_t)k * N + o) * vs_stride + c0 + lane] = mine;
    }
  }
  if (B != nullptr) {
    CT mine = 0;
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
      const CT t = wave_sum(bacc[c]);
      if (lane == c) mine = t;
    }
    const int c = c0 + lane;
    if (lane < CPL && c < C) {
      const int q = c / 3, chn = c - 3 * q;
      B[((int64_t)q * N + perm[o]) * 3 + chn] = mine;
    }
  }
}

template <typename VT, typename CT, int CPL>
static hipError_t transport_launch(const int32_t *col, const void *val, int64_t n_keep, int K,
                                   int N, const void *ehat, int Cs, int C, const void *gcol,
                                   const int32_t *perm, void *B, void *vsave, int vs_stride,
                                   int n_chunks, hipStream_t st) {
  constexpr int U = CPL <= 4 ? 4 : (CPL <= 8 ? 2 : 1);
  const int lb = (N + 3) / 4;
  const int hw = ((lb + 7) / 8) * 8;
  hipLaunchKernelGGL((k_transport<VT, CT, CPL, U>), dim3(hw, n_chunks), dim3(256), 0, st, col,
                     (const VT *)val, n_keep, K, N, (const CT *)ehat, Cs, C, (const CT *)gcol,
                     perm, (CT *)B, (CT *)vsave, vs_stride, lb);
  return hipGetLastError();
}

#define TLT_CPL_LIST(X) X(4) X(8) X(12) X(16) X(24) X(28) X(32) X(36) X(48) X(64)

bool transport_cpl_supported(int cpl, bool fp64) {
  switch (cpl) {
#define CASE(n) case n: return true;
    TLT_CPL_LIST(CASE)
#undef CASE
    default: return false;
  }
}

template <typename VT, typename CT>
static hipError_t transport_dispatch(int cpl, const int32_t *col, const void *val, int64_t n_keep,
                                     int K, int N, const void *ehat, int Cs, int C,
                                     const void *gcol, const int32_t *perm, void *B, void *vsave,
                                     int vs_stride, hipStream_t st) {
  const int n_chunks = (C + cpl - 1) / cpl;
  switch (cpl) {
#define CASE(n)                                                                                \
  case n:                                                                                      \
    return transport_launch<VT, CT, n>(col, val, n_keep, K, N, ehat, Cs, C, gcol, perm, B,     \
                                       vsave, vs_stride, n_chunks, st);
    TLT_CPL_LIST(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_transport(const int32_t *col, const void *val, int vdt, int64_t n_keep, int K,
                            int N, const void *ehat, int Cs, int C, int cpl, const void *gcol,
                            const int32_t *perm, void *B, void *vsave, int vs_stride, bool fp64,
                            hipStream_t st) {
  if (fp64) {
    if (vdt != 0) return hipErrorInvalidValue;
    return transport_dispatch<double, double>(cpl, col, val, n_keep, K, N, ehat, Cs, C, gcol,
                                              perm, B, vsave, vs_stride, st);
  }
  switch (vdt) {
    case 1: return transport_dispatch<float, float>(cpl, col, val, n_keep, K, N, ehat, Cs, C, gcol, perm, B, vsave, vs_stride, st);
    case 2: return transport_dispatch<bf16s, float>(cpl, col, val, n_keep, K, N, ehat, Cs, C, gcol, perm, B, vsave, vs_stride, st);
    case 3: return transport_dispatch<f16s, float>(cpl, col, val, n_keep, K, N, ehat, Cs, C, gcol, perm, B, vsave, vs_stride, st);
    default: return hipErrorInvalidValue;
  }
}

// Material-only update (Steps 3-4 of Sec. 4): B = sum_k g_k v_k from the
// v_k saved by the last full render.  One thread per (vertex, column).
template <typename CT>
__global__ __launch_bounds__(256) void k_combine(const CT *__restrict__ V, int Cs,
                                                 const CT *__restrict__ gcol, int K, int N, int C,
                                                 const int32_t *__restrict__ perm,
                                                 CT *__restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)N * C) return;
  const int o = (int)(t / C), c = (int)(t - (int64_t)o * C);
  CT s = 0;
  for (int k = 0; k < K; ++k) s = fma(gcol[(size_t)k * Cs + c], V[((int64_t)k * N + o) * Cs + c], s);
  const int q = c / 3, ch = c - 3 * q;
  B[((int64_t)q * N + perm[o]) * 3 + ch] = s;
}

hipError_t launch_combine(const void *V, int Cs, const void *gcol, int K, int N, int C,
                          const int32_t *perm, void *B, bool fp64, hipStream_t st) {
  const int64_t n = (int64_t)N * C;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (fp64)
    hipLaunchKernelGGL(k_combine<double>, dim3(blocks), dim3(256), 0, st, (const double *)V, Cs,
                       (const double *)gcol, K, N, C, perm, (double *)B);
  else
    hipLaunchKernelGGL(k_combine<float>, dim3(blocks), dim3(256), 0, st, (const float *)V, Cs,
                       (const float *)gcol, K, N, C, perm, (float *)B);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// a6: adjoint.
//
//   gbar[k][c]  = sum_o dB[c](perm[o]) * V[k][o][c]
//   X[c][lm]    = sum_o dB[c](perm[o]) * sum_k g[k][c] P[k][o][lm]
// Stage 1: one thread per output value and vertex block (ADJ_VB vertices),
// partial sums to scratch.  Stage 2: fixed-order sum over blocks in float64,
// then thetabar = sum gbar dg and dSH from X.
// ---------------------------------------------------------------------------

constexpr int ADJ_VB = 256;

static size_t adj_red_offset(size_t nblk, size_t nout, bool fp64) {
  return (nblk * nout * (fp64 ? 8 : 4) + 255) / 256 * 256;
}

size_t adjoint_partial_bytes(int N, int K, int n_sh, int C, bool fp64) {
  const size_t nblk = (N + ADJ_VB - 1) / ADJ_VB;
  const size_t nout = (size_t)K * C + (size_t)C * n_sh;
  return adj_red_offset(nblk, nout, fp64) + nout * 8;
}

template <typename CT>
__global__ __launch_bounds__(256) void k_adj_partial(
    const CT *__restrict__ dB, const CT *__restrict__ V, int Cs, const CT *__restrict__ P,
    int Psh, const CT *__restrict__ gcol, const int32_t *__restrict__ perm, int N, int K, int n_sh,
    int C, CT *__restrict__ part) {
  const int t = blockIdx.y * 256 + threadIdx.x;
  const int n_g = K * C, n_x = C * n_sh;
  if (t >= n_g + n_x) return;
  const int o0 = blockIdx.x * ADJ_VB;
  const int o1 = min(N, o0 + ADJ_VB);
  CT acc = 0;
  if (t < n_g) {
    const int k = t / C, c = t - k * C;
    const int q = c / 3, ch = c - 3 * q;
    for (int o = o0; o < o1; ++o) {
      const CT d = dB[((int64_t)q * N + perm[o]) * 3 + ch];
      acc = fma(d, V[((int64_t)k * N + o) * Cs + c], acc);
    }
  } else {
    const int u = t - n_g;
    const int c = u / n_sh, lm = u - c * n_sh;
    const int q = c / 3, ch = c - 3 * q;
    for (int o = o0; o < o1; ++o) {
      const CT d = dB[((int64_t)q * N + perm[o]) * 3 + ch];
      CT s = 0;
      for (int k = 0; k < K; ++k) s = fma(gcol[(size_t)k * Cs + c], P[((int64_t)k * N + o) * Psh + lm], s);
      acc = fma(d, s, acc);
    }
  }
  part[(size_t)blockIdx.x * (n_g + n_x) + t] = acc;
}

template <typename CT>
__global__ __launch_bounds__(256) void k_adj_reduce(const CT *__restrict__ part, int nblk, int nout,
                                                    double *__restrict__ out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= nout) return;
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += (double)part[(size_t)b * nout + t];
  out[t] = s;
}

// thetabar[m][ch][p] and dSH[l][lm][ch] from the reduced sums.
template <typename CT>
__global__ void k_adj_out(const double *__restrict__ red, const double *__restrict__ dg64, int K,
                          int n_sh, Cols cols, CT *__restrict__ dSH, double *__restrict__ dTheta) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = cols.C;
  const double *gbar = red;             // [K][C]
  const double *X = red + (size_t)K * C; // [C][n_sh]
  const int n_th = cols.n_mat * 9;
  const int n_l = cols.n_light * n_sh * 3;
  if (t < n_th) {
    const int m = t / 9, ch = (t / 3) % 3, p = t % 3;
    double s = 0.0;
    for (int q = 0; q < cols.n_out; ++q) {
      const int mq = cols.n_mat > 1 ? q : 0;
      if (mq != m) continue;
      const int c = 3 * q + ch;
      for (int k = 0; k < K; ++k) s += gbar[(size_t)k * C + c] * dg64[(((size_t)m * 3 + ch) * K + k) * 3 + p];
    }
    dTheta[t] = s;
  } else if (t < n_th + n_l) {
    const int u = t - n_th;
    const int l = u / (n_sh * 3), lm = (u / 3) % n_sh, ch = u % 3;
    double s = 0.0;
    for (int q = 0; q < cols.n_out; ++q) {
      const int lq = cols.n_light > 1 ? q : 0;
      if (lq != l) continue;
      s += X[(size_t)(3 * q + ch) * n_sh + lm];
    }
    dSH[u] = (CT)s;
  }
}

hipError_t launch_adjoint(const void *dB, const void *V, int Cs, const void *P, int Psh,
                          const void *gcol, const double *dg64, const int32_t *perm, int N, int K,
                          int n_sh, Cols cols, bool fp64, void *partial, size_t partial_bytes,
                          void *dSH, double *dTheta, hipStream_t st) {
  const int C = cols.C;
  const int nblk = (N + ADJ_VB - 1) / ADJ_VB;
  const int nout = K * C + C * n_sh;
  if (partial_bytes < adjoint_partial_bytes(N, K, n_sh, C, fp64)) return hipErrorInvalidValue;
  double *red = (double *)((char *)partial + adj_red_offset(nblk, nout, fp64));
  const dim3 g1(nblk, (nout + 255) / 256);
  const int n_fin = cols.n_mat * 9 + cols.n_light * n_sh * 3;
  if (fp64) {
    hipLaunchKernelGGL(k_adj_partial<double>, g1, dim3(256), 0, st, (const double *)dB,
                       (const double *)V, Cs, (const double *)P, Psh, (const double *)gcol, perm,
                       N, K, n_sh, C, (double *)partial);
    hipLaunchKernelGGL(k_adj_reduce<double>, dim3((nout + 255) / 256), dim3(256), 0, st,
                       (const double *)partial, nblk, nout, red);
    hipLaunchKernelGGL(k_adj_out<double>, dim3((n_fin + 255) / 256), dim3(256), 0, st, red, dg64,
                       K, n_sh, cols, (double *)dSH, dTheta);
  } else {
    hipLaunchKernelGGL(k_adj_partial<float>, g1, dim3(256), 0, st, (const float *)dB,
                       (const float *)V, Cs, (const float *)P, Psh, (const float *)gcol, perm, N,
                       K, n_sh, C, (float *)partial);
    hipLaunchKernelGGL(k_adj_reduce<float>, dim3((nout + 255) / 256), dim3(256), 0, st,
                       (const float *)partial, nblk, nout, red);
    hipLaunchKernelGGL(k_adj_out<float>, dim3((n_fin + 255) / 256), dim3(256), 0, st, red, dg64,
                       K, n_sh, cols, (float *)dSH, dTheta);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Storage conversion (load time): float64 -> float64/float32/bf16/f16, each
// rounded to nearest even (16-bit types via float32).
// ---------------------------------------------------------------------------

__device__ inline uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__global__ void k_quantize(const double *__restrict__ src, void *__restrict__ dst, int vdt,
                           int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = src[i];
  switch (vdt) {
    case 0: ((double *)dst)[i] = v; break;
    case 1: ((float *)dst)[i] = (float)v; break;
    case 2: ((uint16_t *)dst)[i] = to_bf16((float)v); break;
    default: ((uint16_t *)dst)[i] = __builtin_bit_cast(uint16_t, (_Float16)(float)v); break;
  }
}

hipError_t launch_quantize(const double *src, void *dst, int vdt, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_quantize, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, vdt, n);
  return hipGetLastError();
}

}  // namespace tlt
