// Per-frame preparation in ONE launch (heterogeneous workgroups):
//
//   [0, n_gk)              material weights g_k and dg_k/dtheta (float64),
//                              rendering Step 3 of Sec. 4 with Eq. (4);
//   [n_gk, n_gk + n_tl)    E = T L on MFMA, times area, Haar levels
//                              inside a 256-row chunk (Step 1, Eq. 6 and 8);
//   [.., + n_zero)         clears B at the vertices whose rows the
//                              transport kernel splits between two waves.
//
// A second small launch (k_haar_top) runs the coarse Haar levels over the
// chunk sums.
//
// MFMA 16x16x4 operand layout (f32 and f64 alike): lane l supplies
// A[l%16][l/16] and B[l/16][l%16].  Result element v of lane l is
// D[4*(l/16)+v][l%16] for f32 but D[(l/16)+4v][l%16] for f64 (checked on
// gfx950 with a probe of known operands).

#include <algorithm>

#include "device_common.h"

namespace tlt {

// ---------------------------------------------------------------------------
// Material weights: dipole R_d (Eq. 4) with its parameter derivatives.
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

__device__ void gk_block(const PrepArgs &a, int mc, double *smem) {
  // smem: q[4][nr] (R_d and its three partials on the nodes), red[K][4],
  // bs[K][nr] (the basis, staged once)
  double *q = smem;
  double *red = smem + 4 * (size_t)a.nr;
  double *bs = red + 4 * (size_t)a.K;
  const int m = mc / 3, ch = mc % 3;
  const double sa = a.theta[mc * 3 + 0], ss = a.theta[mc * 3 + 1], eta = a.theta[mc * 3 + 2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // Validation of the material (read here, not on the host): the dipole of
  // Eq. (4) needs sigma_a, sigma_s' > 0 and the F_dr fit eta >= 1, all
  // finite.  An invalid channel gets NaN weights (its radiance is NaN, never
  // silently wrong) and raises the context's invalid flag; a valid one
  // outside the PCA table's range raises the range flag (still computed).
  const bool bad = !(isfinite(sa) && isfinite(ss) && isfinite(eta) && sa > 0.0 && ss > 0.0 && eta >= 1.0);
  const bool far = !bad && a.has_range &&
                   (sa < a.mat_lo[0] || sa > a.mat_hi[0] || ss < a.mat_lo[1] || ss > a.mat_hi[1] ||
                    eta < a.mat_lo[2] || eta > a.mat_hi[2]);
  if (threadIdx.x == 0 && a.mstat != nullptr) {
    if (bad) {
      a.mstat[0] = 1;
      a.mstat[2] = mc;
    }
    if (far) a.mstat[1] = 1;
  }
  // the basis is staged in LDS when it fits the budget (else it is read from
  // memory in place).  With one node per thread (n_r <= 256, K <= 16) the
  // thread's basis values are loaded into registers first and stored after
  // the dipole work, so the loads complete under it.
  const double *bsrc = a.gk_stage ? bs : a.basis;
  if (a.gk_stage && a.nr <= 256 && a.K <= 16) {
    const int n = threadIdx.x;
    double breg[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) breg[k] = (k < a.K && n < a.nr) ? a.basis[(size_t)k * a.nr + n] : 0.0;
    if (n < a.nr) {
      const RdGrad g = rd_grad(a.rn[n], sa, ss, eta);
      q[n] = g.R;
      q[a.nr + n] = g.da;
      q[2 * a.nr + n] = g.ds;
      q[3 * a.nr + n] = g.de;
    }
#pragma unroll
    for (int k = 0; k < 16; ++k)
      if (k < a.K && n < a.nr) bs[(size_t)k * a.nr + n] = breg[k];
  } else {
    if (a.gk_stage)
      for (int i = threadIdx.x; i < a.K * a.nr; i += 256) bs[i] = a.basis[i];
    for (int n = threadIdx.x; n < a.nr; n += 256) {
      const RdGrad g = rd_grad(a.rn[n], sa, ss, eta);
      q[n] = g.R;
      q[a.nr + n] = g.da;
      q[2 * a.nr + n] = g.ds;
      q[3 * a.nr + n] = g.de;
    }
  }
  __syncthreads();
  // projections on b_k (Sec. 2.2): wave w takes quantity w (R_d or one of
  // its partials) for eight terms at a time; lanes sum over the nodes in a
  // fixed order, then the eight wave sums run side by side
  for (int k0 = 0; k0 < a.K; k0 += 8) {
    double p[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) p[j] = 0.0;
    for (int n = lane; n < a.nr; n += 64) {
      const double qv = q[wave * a.nr + n];
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (k0 + j < a.K) p[j] = fma(qv, bsrc[(size_t)(k0 + j) * a.nr + n], p[j]);
    }
#pragma unroll
    for (int j = 0; j < 8; ++j) p[j] = wave_sum(p[j]);
    if (lane == 0) {
#pragma unroll
      for (int j = 0; j < 8; ++j)
        if (k0 + j < a.K) red[(size_t)(k0 + j) * 4 + wave] = p[j];
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < 4 * a.K; t += 256) {
    const int k = t / 4, qn = t % 4;
    const double acc = bad ? __builtin_nan("") : red[t];
    if (qn == 0) {
      a.g64[(size_t)mc * a.K + k] = acc;
      for (int o = 0; o < a.cols.n_out; ++o) {
        const int mo = a.cols.n_mat > 1 ? o : 0;
        if (mo != m) continue;
        const int c = 3 * o + ch;
        if (a.fp64)
          ((double *)a.gcol)[(size_t)k * a.Cs + c] = acc;
        else
          ((float *)a.gcol)[(size_t)k * a.Cs + c] = (float)acc;
      }
    } else {
      a.dg64[((size_t)mc * a.K + k) * 3 + (qn - 1)] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// Irradiance E = T L, area weight and the Haar levels inside a chunk.
// ---------------------------------------------------------------------------

constexpr int TL_CH = 256;
constexpr int TL_STRIDE = 17;

// Irradiance store: float Ehat and, for 16-bit transport tiles, its split
// into a high 16-bit part and the 16-bit rounding of the remainder, packed
// as (hi | lo << 16), so the tile kernel gathers one word per element.
__device__ __forceinline__ uint32_t split16(float x, int kind) {
  if (kind == 1) {
    const __bf16 hi = (__bf16)x;
    const __bf16 lo = (__bf16)(x - (float)hi);
    return (uint32_t)__builtin_bit_cast(uint16_t, hi) | ((uint32_t)__builtin_bit_cast(uint16_t, lo) << 16);
  }
  const _Float16 hi = (_Float16)x;
  const _Float16 lo = (_Float16)(x - (float)hi);
  return (uint32_t)__builtin_bit_cast(uint16_t, hi) | ((uint32_t)__builtin_bit_cast(uint16_t, lo) << 16);
}

template <typename CT>
__device__ __forceinline__ void store_e(CT *ehat, uint32_t *ehat2, int split, size_t idx, CT v) {
  ehat[idx] = v;
  if constexpr (sizeof(CT) == 4) {
    if (ehat2 != nullptr) ehat2[idx] = split16(v, split);
  }
}

// Haar levels of one chunk with R = ch_rows / 16 rows per thread: thread
// (g = threadIdx.x / 16, column cc = threadIdx.x % 16) takes rows g R ..
// g R + R - 1 of its column into registers and runs the log2 R levels whose
// pairs lie inside them without any barrier; the 16 sums per column left
// then go through LDS once, and one thread per column runs the last four
// levels.  Every detail and sum is the same expression of the same two
// values as in the level-by-level form, so the results are identical.
template <int R, typename CT>
__device__ void haar_chunk(const PrepArgs &a, CT *x, int chunk, int c0, CT *ehat, uint32_t *ehat2,
                           CT *partial) {
  const CT h = CT(0.70710678118654752440);
  const int cc = threadIdx.x & 15, g = threadIdx.x >> 4;
  CT v[R];
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = x[(g * R + r) * TL_STRIDE + cc];
  int half = a.ch_rows >> 1;
#pragma unroll
  for (int n = R; n > 1; n >>= 1) {
#pragma unroll
    for (int p = 0; p < n / 2; ++p) {
      const CT lo = v[2 * p], hi = v[2 * p + 1];
      const int64_t j = idx::haar_row(half, a.n_chunks, chunk, idx::haar_reg_detail(g, n, p));
      store_e(ehat, ehat2, a.split, (size_t)j * a.Cs + c0 + cc, (lo - hi) * h);
      v[p] = (lo + hi) * h;
    }
    half >>= 1;
  }
  __syncthreads();  // every thread has read its rows of x
  x[g * TL_STRIDE + cc] = v[0];
  __syncthreads();
  if (g != 0) return;
  CT u[16];
#pragma unroll
  for (int r = 0; r < 16; ++r) u[r] = x[r * TL_STRIDE + cc];
#pragma unroll
  for (int n = 16; n > 1; n >>= 1) {
#pragma unroll
    for (int p = 0; p < n / 2; ++p) {
      const CT lo = u[2 * p], hi = u[2 * p + 1];
      const int64_t j = idx::haar_row(half, a.n_chunks, chunk, p);
      store_e(ehat, ehat2, a.split, (size_t)j * a.Cs + c0 + cc, (lo - hi) * h);
      u[p] = (lo + hi) * h;
    }
    half >>= 1;
  }
  if (a.n_chunks == 1)
    store_e(ehat, ehat2, a.split, (size_t)c0 + cc, u[0]);
  else
    partial[(size_t)chunk * a.Cs + c0 + cc] = u[0];
}

template <typename TT, typename CT>
__device__ void tl_block(const PrepArgs &a, int t, unsigned char *smem) {
  typedef typename MfmaOut<CT>::V4 V4;
  // LDS: x [TL_CH][TL_STRIDE] (E, then the Haar levels), Ts [ch_rows *
  // n_sh] (the chunk's transfer rows, contiguous as in T), Ls [n_shp][16]
  // (lighting columns of the tile), As [ch_rows] (areas)
  CT *x = reinterpret_cast<CT *>(smem);
  TT *Ts = reinterpret_cast<TT *>(x + TL_CH * TL_STRIDE);   // storage type, as in T
  const int t_ld = a.t_ld ? a.t_ld : a.n_sh;               // row stride of T
  CT *Ls = reinterpret_cast<CT *>(Ts + ((size_t)a.ch_rows * t_ld + 15) / 16 * 16);
  CT *As = Ls + (size_t)a.n_shp * 16;
  const int chunk = t % a.n_chunks;
  const int ctile = t / a.n_chunks;
  const int c0 = ctile * 16;
  const int i0 = chunk * a.ch_rows;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const TT *T = (const TT *)a.T;
  const CT *sh = (const CT *)a.sh;
  const CT *area = (const CT *)a.area;
  CT *ehat = (CT *)a.ehat;
  uint32_t *ehat2 = (uint32_t *)a.ehat2;
  CT *partial = (CT *)a.partial;

  const int nr_e = max(0, min(a.ch_rows, (a.t_rows ? a.t_rows : a.N) - i0));
  if (a.E != nullptr) {
    // supplied irradiance: E at the chunk's vertices (gathered through the
    // Morton permutation) times the area, in place of T L
    const CT *E = (const CT *)a.E;
    for (int idx = threadIdx.x; idx < a.ch_rows * 16; idx += 256) {
      const int lr = idx >> 4, n = idx & 15, c = c0 + n;
      CT v = 0;
      if (lr < nr_e && c < a.cols.C) {
        const int q = c / 3, ch = c - 3 * q;
        const int l = a.cols.n_light > 1 ? q : 0;
        const int64_t o = a.perm[i0 + lr];
        v = E[((int64_t)l * a.N + o) * 3 + ch] * area[i0 + lr];
      }
      x[lr * TL_STRIDE + n] = v;
    }
  }
  // Stage everything the chunk reads with one batch of loads.  The chunk's
  // transfer rows are one contiguous range of T, read as 16-byte vectors
  // through a buffer resource (reads past the end of T return zeros), all
  // issued before any is used.
  const int nr = nr_e;                                      // real vertices of the chunk
  if (a.E == nullptr) {
    constexpr int TSZ = sizeof(TT), VEC = 16 / TSZ, VPT = 8;
    const int nel = nr * t_ld;                              // elements of the chunk
    const int nvec = (nel + VEC - 1) / VEC;
    const __amdgpu_buffer_rsrc_t trs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)((const char *)T + (size_t)i0 * t_ld * TSZ), (short)0, nel * TSZ, 0x00020000);
    for (int v0 = 0; v0 < nvec; v0 += 256 * VPT) {
      uint4 buf[VPT];
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const int v = v0 + u * 256 + threadIdx.x;
        buf[u] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                               trs, v < nvec ? v * 16 : nel * TSZ, 0, 0));
      }
#pragma unroll
      for (int u = 0; u < VPT; ++u) {
        const int v = v0 + u * 256 + threadIdx.x;
        if (v < nvec) reinterpret_cast<uint4 *>(Ts)[v] = buf[u];
      }
    }
    for (int idx = threadIdx.x; idx < a.n_shp * 16; idx += 256) {
      const int kc = idx >> 4, n = idx & 15, c = c0 + n;
      CT b = 0;
      if (kc < a.n_sh) {
        if (sh == nullptr) {
          b = (kc == c) ? CT(1) : CT(0);
        } else if (c < a.cols.C) {
          const int q = c / 3, ch = c - 3 * q;
          const int l = a.cols.n_light > 1 ? q : 0;
          b = sh[((size_t)l * a.n_sh + kc) * 3 + ch];
        }
      }
      Ls[idx] = b;
    }
    // no area: rows that carry it already (the folded G = H (A o T))
    for (int idx = threadIdx.x; idx < a.ch_rows; idx += 256)
      As[idx] = idx < nr ? (area ? area[i0 + idx] : CT(1)) : CT(0);
  }
  __syncthreads();
  if (a.E == nullptr && 64 * wave < a.ch_rows) {
    V4 acc[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) acc[u] = V4{0, 0, 0, 0};
    for (int kk = 0; kk < a.n_shp; kk += 4) {
      const int kc = kk + lk;
      const CT b = Ls[kc * 16 + li];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int lr = 64 * wave + 16 * u + li;
        // rows past the last vertex (zero padding) and columns past n_sh
        // were never staged: they contribute zeros
        const CT av = (lr < nr && kc < a.n_sh) ? ld<TT, CT>(Ts, lr * t_ld + kc) : CT(0);
        acc[u] = mfma16(av, b, acc[u]);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int lr = 64 * wave + 16 * u + MfmaOut<CT>::row(lk, v);
        if (lr < a.ch_rows) x[lr * TL_STRIDE + li] = acc[u][v] * As[lr];
      }
    }
  }
  __syncthreads();

  if (!a.haar) {
    for (int idx = threadIdx.x; idx < a.ch_rows * 16; idx += 256) {
      const int lr = idx >> 4, cc = idx & 15;
      const int r = i0 + lr;
      if (r < a.n_rows) store_e(ehat, ehat2, a.split, (size_t)r * a.Cs + c0 + cc, x[lr * TL_STRIDE + cc]);
    }
    return;
  }

  switch (a.ch_rows) {
    case 16: haar_chunk<1, CT>(a, x, chunk, c0, ehat, ehat2, partial); return;
    case 32: haar_chunk<2, CT>(a, x, chunk, c0, ehat, ehat2, partial); return;
    case 64: haar_chunk<4, CT>(a, x, chunk, c0, ehat, ehat2, partial); return;
    case 128: haar_chunk<8, CT>(a, x, chunk, c0, ehat, ehat2, partial); return;
    case 256: haar_chunk<16, CT>(a, x, chunk, c0, ehat, ehat2, partial); return;
    default: break;
  }
  const CT h = CT(0.70710678118654752440);
  for (int len = a.ch_rows; len > 1; len >>= 1) {
    const int half = len >> 1;
    CT sv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = threadIdx.x + 256 * u;
      if (idx < half * 16) {
        const int i = idx >> 4, cc = idx & 15;
        const CT p = x[(2 * i) * TL_STRIDE + cc];
        const CT q = x[(2 * i + 1) * TL_STRIDE + cc];
        const int64_t j = idx::haar_row(half, a.n_chunks, chunk, i);
        store_e(ehat, ehat2, a.split, (size_t)j * a.Cs + c0 + cc, (p - q) * h);
        sv[u] = (p + q) * h;
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int idx = threadIdx.x + 256 * u;
      if (idx < half * 16) x[(idx >> 4) * TL_STRIDE + (idx & 15)] = sv[u];
    }
    __syncthreads();
  }
  if (a.n_chunks == 1) {
    if (threadIdx.x < 16) store_e(ehat, ehat2, a.split, (size_t)c0 + threadIdx.x, x[threadIdx.x]);
    return;
  }
  if (threadIdx.x < 16) partial[(size_t)chunk * a.Cs + c0 + threadIdx.x] = x[threadIdx.x];
}

// Coarse Haar levels over the n_chunks chunk sums of one column (a second,
// small launch: the chunk sums come from every XCD, and a kernel boundary
// is the cheap way to make them visible).  grid: Cs workgroups.
template <typename CT>
__global__ __launch_bounds__(256) void k_haar_top(const CT *__restrict__ partial, int n_chunks,
                                                  int Cs, CT *__restrict__ ehat,
                                                  uint32_t *__restrict__ ehat2, int split) {
  extern __shared__ __align__(16) unsigned char raw[];
  CT *s0 = reinterpret_cast<CT *>(raw);
  CT *s1 = s0 + n_chunks;
  const int c = blockIdx.x;
  for (int i = threadIdx.x; i < n_chunks; i += 256) s0[i] = partial[(size_t)i * Cs + c];
  __syncthreads();
  const CT h = CT(0.70710678118654752440);
  CT *src = s0, *dst = s1;
  for (int len = n_chunks; len > 1; len >>= 1) {
    const int half = len >> 1;
    for (int i = threadIdx.x; i < half; i += 256) {
      const CT p = src[2 * i], q = src[2 * i + 1];
      // the levels above the chunks run as one chunk of n_chunks values
      store_e(ehat, ehat2, split, (size_t)idx::haar_row(half, 1, 0, i) * Cs + c, (p - q) * h);
      dst[i] = (p + q) * h;
    }
    __syncthreads();
    CT *t = src;
    src = dst;
    dst = t;
  }
  if (threadIdx.x == 0) store_e(ehat, ehat2, split, (size_t)c, src[0]);
}

template <typename CT>
__device__ void zero_block(const PrepArgs &a, int t) {
  CT *B = (CT *)a.B;
  const int64_t n = (int64_t)a.n_zero * a.cols.C;
  for (int64_t idx = (int64_t)t * 256 + threadIdx.x; idx < n; idx += (int64_t)a.n_zero_blocks * 256) {
    const int v = (int)(idx / a.cols.C), c = (int)(idx % a.cols.C);
    const int q = c / 3, ch = c - 3 * q;
    B[((int64_t)q * a.N + a.zero_v[v]) * 3 + ch] = CT(0);
  }
}

template <typename TT, typename CT>
__global__ __launch_bounds__(256) void k_prep(PrepArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  int b = blockIdx.x;
  if (b < a.n_gk_blocks) {
    gk_block(a, b, reinterpret_cast<double *>(smem));
    return;
  }
  b -= a.n_gk_blocks;
  if (b < a.n_tl_blocks) {
    tl_block<TT, CT>(a, b, smem);
    return;
  }
  b -= a.n_tl_blocks;
  zero_block<CT>(a, b);
}

size_t prep_lds_bytes(const PrepArgs &a) {
  const size_t esz = a.fp64 ? 8 : 4;
  size_t s = sizeof(double) * (4 * (size_t)a.nr + 4 * (size_t)a.K +
                               (a.gk_stage ? (size_t)a.K * a.nr : 0));             // weights
  if (a.n_tl_blocks > 0)
    s = std::max(s, esz * ((size_t)TL_CH * TL_STRIDE + (size_t)a.n_shp * 16 + (size_t)a.ch_rows) +
                        ((size_t)a.ch_rows * (a.t_ld ? a.t_ld : a.n_sh) + 15) / 16 * 16 *
                            (a.tdt == 0 ? 8 : a.tdt == 1 ? 4 : 2));
  return s;
}

hipError_t launch_prep(const PrepArgs &a, hipStream_t st) {
  const int blocks = a.n_gk_blocks + a.n_tl_blocks + a.n_zero_blocks;
  if (blocks == 0) return hipSuccess;
  const size_t lds = prep_lds_bytes(a);
  if (a.fp64) {
    if (a.tdt != 0) return hipErrorInvalidValue;
    TLT_LAUNCH((k_prep<double, double>), dim3(blocks), dim3(256), lds, st, a);
  } else {
    switch (a.tdt) {
      case 1: TLT_LAUNCH((k_prep<float, float>), dim3(blocks), dim3(256), lds, st, a); break;
      case 2: TLT_LAUNCH((k_prep<bf16s, float>), dim3(blocks), dim3(256), lds, st, a); break;
      case 3: TLT_LAUNCH((k_prep<f16s, float>), dim3(blocks), dim3(256), lds, st, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.n_tl_blocks > 0 && a.haar && a.n_chunks > 1) {
    const size_t lds2 = (size_t)a.n_chunks * 3 / 2 * (a.fp64 ? 8 : 4);
    if (a.fp64)
      TLT_LAUNCH((k_haar_top<double>), dim3(a.Cs), dim3(256), lds2, st,
                         (const double *)a.partial, a.n_chunks, a.Cs, (double *)a.ehat,
                         (uint32_t *)nullptr, 0);
    else
      TLT_LAUNCH((k_haar_top<float>), dim3(a.Cs), dim3(256), lds2, st,
                         (const float *)a.partial, a.n_chunks, a.Cs, (float *)a.ehat,
                         (uint32_t *)a.ehat2, a.split);
    e = hipGetLastError();
  }
  return e;
}

}  // namespace tlt
