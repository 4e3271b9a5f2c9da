// Small kernels: material-only combine, adjoint reductions, storage
// conversion at load time.

#include "device_common.h"

namespace tlt {

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
// Adjoint of the transport.
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
