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

// Float32 form: one thread per vertex and four consecutive columns (Cs is a
// multiple of 16), the KT <= 16 terms' 16-byte loads of v_k all issued
// before the sums, so each thread keeps KT loads in flight.
template <int KT>
__global__ __launch_bounds__(256) void k_combine4(const float *__restrict__ V, int Cs,
                                                  const float *__restrict__ gcol, int K, int N, int C,
                                                  const int32_t *__restrict__ perm,
                                                  float *__restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int nq = Cs / 4;
  if (t >= (int64_t)N * nq) return;
  const int o = (int)(t / nq), c0 = 4 * (int)(t - (int64_t)o * nq);
  if (c0 >= C) return;
  float4 v[KT], g[KT];
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    const int kk = min(k, K - 1);
    v[k] = *reinterpret_cast<const float4 *>(V + ((int64_t)kk * N + o) * Cs + c0);
    g[k] = *reinterpret_cast<const float4 *>(gcol + (size_t)kk * Cs + c0);
  }
  float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int k = 0; k < KT; ++k) {
    if (k < K) {
      s[0] = fmaf(g[k].x, v[k].x, s[0]);
      s[1] = fmaf(g[k].y, v[k].y, s[1]);
      s[2] = fmaf(g[k].z, v[k].z, s[2]);
      s[3] = fmaf(g[k].w, v[k].w, s[3]);
    }
  }
  const int64_t po = perm[o];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int c = c0 + j;
    if (c < C) {
      const int q = c / 3, ch = c - 3 * q;
      B[((int64_t)q * N + po) * 3 + ch] = s[j];
    }
  }
}

// Outgoing Fresnel factor of Eq. (3)/(6): B[q][perm[o]][ch] *= (1/pi)
// F_t(eta[mat(q)][ch], w_o(o)), from cos(w_o, n) per Morton position (0 or
// less: seen from behind, factor 0).  Unpolarised dielectric transmittance,
// air outside, index eta inside.
template <typename CT>
__global__ __launch_bounds__(256) void k_view(CT *__restrict__ B, const CT *__restrict__ cosv,
                                              const double *__restrict__ theta, Cols cols, int N,
                                              const int32_t *__restrict__ perm) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)cols.n_out * N * 3) return;
  const int ch = (int)(t % 3);
  const int64_t r = t / 3;
  const int o = (int)(r % N), q = (int)(r / N);
  const int m = cols.n_mat > 1 ? q : 0;
  const CT eta = (CT)theta[((size_t)m * 3 + ch) * 3 + 2];
  const CT c = cosv[o];
  CT f = 0;
  if (c > CT(0)) {
    const CT cc = c < CT(1) ? c : CT(1);
    const CT ct = sqrt(CT(1) - (CT(1) - cc * cc) / (eta * eta));
    const CT rs = (cc - eta * ct) / (cc + eta * ct);
    const CT rp = (eta * cc - ct) / (eta * cc + ct);
    f = (CT(1) - CT(0.5) * (rs * rs + rp * rp)) * CT(0.31830988618379067154);
  }
  B[((int64_t)q * N + perm[o]) * 3 + ch] *= f;
}

hipError_t launch_view(void *B, const void *cosv, const double *theta, Cols cols, int N,
                       const int32_t *perm, bool fp64, hipStream_t st) {
  const int64_t n = (int64_t)cols.n_out * N * 3;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (fp64)
    TLT_LAUNCH(k_view<double>, dim3(blocks), dim3(256), 0, st, (double *)B, (const double *)cosv, theta,
               cols, N, perm);
  else
    TLT_LAUNCH(k_view<float>, dim3(blocks), dim3(256), 0, st, (float *)B, (const float *)cosv, theta,
               cols, N, perm);
  return hipGetLastError();
}

hipError_t launch_combine(const void *V, int Cs, const void *gcol, int K, int N, int C,
                          const int32_t *perm, void *B, bool fp64, hipStream_t st) {
  const int64_t n = (int64_t)N * C;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (fp64)
    TLT_LAUNCH(k_combine<double>, dim3(blocks), dim3(256), 0, st, (const double *)V, Cs,
                       (const double *)gcol, K, N, C, perm, (double *)B);
  else if (Cs % 16 == 0 && K <= 16) {
    const int64_t n4 = (int64_t)N * (Cs / 4);
    const unsigned b4 = (unsigned)((n4 + 255) / 256);
    if (K <= 4)
      TLT_LAUNCH(k_combine4<4>, dim3(b4), dim3(256), 0, st, (const float *)V, Cs, (const float *)gcol, K,
                 N, C, perm, (float *)B);
    else if (K <= 8)
      TLT_LAUNCH(k_combine4<8>, dim3(b4), dim3(256), 0, st, (const float *)V, Cs, (const float *)gcol, K,
                 N, C, perm, (float *)B);
    else
      TLT_LAUNCH(k_combine4<16>, dim3(b4), dim3(256), 0, st, (const float *)V, Cs, (const float *)gcol,
                 K, N, C, perm, (float *)B);
  } else
    TLT_LAUNCH(k_combine<float>, dim3(blocks), dim3(256), 0, st, (const float *)V, Cs,
                       (const float *)gcol, K, N, C, perm, (float *)B);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Folded lighting transport (Eq. 14, the SH lighting path): with
// P_k = W_k H (A o T) (built at load, [K][N][Psh], Morton rows),
//   B[o, c] = sum_k g_k[c] sum_lm P_k[o, lm] L[light(c)][lm][ch(c)],
// one matrix product over the contraction index (k, lm):
//   B[o, c] = sum_(k,lm) P[o, (k,lm)] Lg[(k,lm), c],  Lg = g_k[c] L[lm][c].
// In exact arithmetic this equals the wavelet transport for the same kept
// coefficients.  Workgroup: 64 rows (one 16-row tile per wave) x up to 64
// columns (FOLD_CG); Lg of the column group is built in LDS; every wave
// reads its P rows directly (one element per lane and step, all loads of a
// term issued before its matrix work).
// ---------------------------------------------------------------------------

constexpr int FOLD_CG = 64;   // columns per workgroup

// Lg[(k, lm)][c] = g_k[c] L[light(c)][lm][ch(c)] (zero past n_sh and C).
template <typename CT>
__global__ __launch_bounds__(256) void k_fold_weights(const CT *__restrict__ gcol, int Cs,
                                                      const CT *__restrict__ sh, Cols cols, int K,
                                                      int Psh, int n_sh, CT *__restrict__ Lg) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  if (i >= K * Psh * Cs) return;
  const int c = i % Cs, kl = i / Cs;
  const int k = kl / Psh, lm = kl - k * Psh;
  CT v = 0;
  if (c < cols.C && lm < n_sh) {
    const int q = c / 3, ch = c - 3 * q;
    const int l = cols.n_light > 1 ? q : 0;
    v = gcol[(size_t)k * Cs + c] * sh[((size_t)l * n_sh + lm) * 3 + ch];
  }
  Lg[i] = v;
}

// Each wave owns FOLD_RT 16-row tiles and FOLD_CG columns.  For each term k
// it holds that term's operands of Lg in registers (read from the small,
// cache-resident Lg) and streams the P_k rows of its tiles: all A operands of
// a term (FOLD_RT x steps values per lane) are requested before the term's
// matrix work.  No LDS, so many waves per compute unit hide the latency.
// NTN real 16-column tiles, MS = Psh / 4 steps, RT tiles per wave: all
// compile-time, so the loads of a term carry no branches (addresses are
// clamped into range and values past the end are zeroed by selects) and
// stay in flight together.
template <typename CT, int NTN, int MS, int RT>
__global__ __launch_bounds__(256) void k_folded(const CT *__restrict__ P, int Psh, int K,
                                                const CT *__restrict__ Lg, int Cs, int C, int N,
                                                const int32_t *__restrict__ perm,
                                                CT *__restrict__ B) {
  typedef typename MfmaOut<CT>::V4 V4;
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int cg0 = blockIdx.y * FOLD_CG;
  const int tile0 = (blockIdx.x * 4 + wave) * RT;       // first 16-row tile of the wave
  V4 acc[RT][NTN];
#pragma unroll
  for (int r = 0; r < RT; ++r)
#pragma unroll
    for (int nt = 0; nt < NTN; ++nt) acc[r][nt] = V4{0, 0, 0, 0};
  const CT *prow[RT];
  bool rok[RT];
#pragma unroll
  for (int r = 0; r < RT; ++r) {
    const int o = (tile0 + r) * 16 + li;
    rok[r] = o < N;
    prow[r] = P + (int64_t)min(o, N - 1) * Psh;
  }
  int bcol[NTN];
#pragma unroll
  for (int nt = 0; nt < NTN; ++nt) bcol[nt] = min(cg0 + nt * 16 + li, Cs - 1);
  for (int k = 0; k < K; ++k) {
    const int64_t koff = (int64_t)k * N * Psh;
    CT av[RT][MS];
    CT bv[MS][NTN];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
      const int lm = 4 * s + lk;   // < Psh: MS * 4 == Psh
#pragma unroll
      for (int r = 0; r < RT; ++r) av[r][s] = prow[r][koff + lm];
      const CT *lrow = Lg + (size_t)(k * Psh + lm) * Cs;
#pragma unroll
      for (int nt = 0; nt < NTN; ++nt) bv[s][nt] = lrow[bcol[nt]];
    }
#pragma unroll
    for (int s = 0; s < MS; ++s)
#pragma unroll
      for (int r = 0; r < RT; ++r)
#pragma unroll
        for (int nt = 0; nt < NTN; ++nt)
          acc[r][nt] = mfma16(rok[r] ? av[r][s] : CT(0), bv[s][nt], acc[r][nt]);
  }
#pragma unroll
  for (int r = 0; r < RT; ++r) {
#pragma unroll
    for (int nt = 0; nt < NTN; ++nt) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = (tile0 + r) * 16 + MfmaOut<CT>::row(lk, v);
        const int c = cg0 + nt * 16 + li;
        if (o < N && c < C) {
          const int q = c / 3, ch = c - 3 * q;
          B[((int64_t)q * N + perm[o]) * 3 + ch] = acc[r][nt][v];
        }
      }
    }
  }
}

// Float32 form with Lg staged in LDS.  The workgroup copies Lg of its
// column group for every term into LDS once (rows padded to FOLD_LDW
// floats, so the four lane groups of a B-operand read hit disjoint banks);
// each wave then streams the P rows of its RT 16-row tiles with 16-byte
// loads, one term ahead of their matrix work.  The contraction over lm is
// taken in a permuted order that makes those loads contiguous: for the
// g-th group of 16 coefficients, lane group lk loads
// P[o][16 g + 4 lk .. 16 g + 4 lk + 3] and its component v enters matrix
// step (g, v) as contraction index 16 g + 4 lk + v; the B operand is read
// from the Lg row of the same index.  The MS % 4 steps left over (Psh not a
// multiple of 16) take one value per lane as in k_folded.
constexpr int FOLD_LDW = FOLD_CG + 4;
constexpr int FOLD_WPB = 8;   // waves per workgroup (they share the staged Lg)

template <int NTN, int MS, int RT>
__global__ __launch_bounds__(FOLD_WPB * 64) void k_folded_lds(const float *__restrict__ P, int Psh,
                                                              int K, const float *__restrict__ Lg,
                                                              int Cs, int C, int N,
                                                              const int32_t *__restrict__ perm,
                                                              float *__restrict__ B) {
  extern __shared__ __align__(16) unsigned char smem[];
  float *lg = reinterpret_cast<float *>(smem);  // [K * Psh][FOLD_LDW]
  constexpr int G4 = MS / 4, R4 = MS % 4;
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int cg0 = blockIdx.y * FOLD_CG;
  f32x4 acc[RT][NTN];
  const float *prow[RT];
  bool rok[RT];
  constexpr int G4n = G4 > 0 ? G4 : 1, R4n = R4 > 0 ? R4 : 1;
  // the A operands of term k (issued one term ahead of their matrix work)
  auto load = [&](int k, float4 (&x4)[RT][G4n], float (&x1)[RT][R4n]) {
    const int64_t koff = (int64_t)k * N * Psh;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
#pragma unroll
      for (int g = 0; g < G4; ++g) x4[r][g] = *reinterpret_cast<const float4 *>(prow[r] + koff + 16 * g + 4 * lk);
#pragma unroll
      for (int q = 0; q < R4; ++q) x1[r][q] = prow[r][koff + 16 * G4 + 4 * q + lk];
    }
  };
  // the B operands of a whole term are read from LDS before its matrix work
  auto compute = [&](int k, const float4 (&x4)[RT][G4n], const float (&x1)[RT][R4n]) {
    const float *lk_rows = lg + (size_t)k * Psh * FOLD_LDW + li;
    float bv[MS][NTN];
#pragma unroll
    for (int g = 0; g < G4; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int nt = 0; nt < NTN; ++nt) bv[4 * g + v][nt] = lk_rows[(16 * g + 4 * lk + v) * FOLD_LDW + nt * 16];
#pragma unroll
    for (int q = 0; q < R4; ++q)
#pragma unroll
      for (int nt = 0; nt < NTN; ++nt) bv[4 * G4 + q][nt] = lk_rows[(16 * G4 + 4 * q + lk) * FOLD_LDW + nt * 16];
#pragma unroll
    for (int g = 0; g < G4; ++g)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int r = 0; r < RT; ++r) {
          const float av = rok[r] ? x4[r][g][v] : 0.f;
#pragma unroll
          for (int nt = 0; nt < NTN; ++nt) acc[r][nt] = mfma16(av, bv[4 * g + v][nt], acc[r][nt]);
        }
#pragma unroll
    for (int q = 0; q < R4; ++q)
#pragma unroll
      for (int r = 0; r < RT; ++r) {
        const float av = rok[r] ? x1[r][q] : 0.f;
#pragma unroll
        for (int nt = 0; nt < NTN; ++nt) acc[r][nt] = mfma16(av, bv[4 * G4 + q][nt], acc[r][nt]);
      }
  };
  float4 a4[RT][G4n], b4[RT][G4n];
  float a1[RT][R4n], b1[RT][R4n];
  // the workgroup stays resident and takes row blocks of 4 RT tiles in
  // turn; the first term of the next block is requested before the
  // current block's stores (and the first block's before the staging)
  const int n_rb = ((N + 15) / 16 + FOLD_WPB * RT - 1) / (FOLD_WPB * RT);
  auto rows = [&](int rb) {
#pragma unroll
    for (int r = 0; r < RT; ++r) {
      const int o = ((rb * FOLD_WPB + wave) * RT + r) * 16 + li;
      rok[r] = o < N;
      prow[r] = P + (int64_t)min(o, N - 1) * Psh;
    }
  };
  rows(blockIdx.x);
  load(0, a4, a1);
  // stage Lg[(k, lm)][cg0 .. cg0 + 63] (zero past Cs; Cs is a multiple of
  // 16): 16-byte items, eight loads in flight per thread
  const int nq = K * Psh * (FOLD_CG / 4);
  constexpr int NTHR = FOLD_WPB * 64;
  for (int i0 = 0; i0 < nq; i0 += NTHR * 8) {
    float4 tmp[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * NTHR + t;
      const int row = i >> 4, col = cg0 + 4 * (i & 15);
      tmp[u] = (i < nq && col < Cs) ? *reinterpret_cast<const float4 *>(Lg + (size_t)row * Cs + col)
                                    : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u * NTHR + t;
      if (i < nq) *reinterpret_cast<float4 *>(lg + (i >> 4) * FOLD_LDW + 4 * (i & 15)) = tmp[u];
    }
  }
  __syncthreads();  // Lg staged
  for (int rb = blockIdx.x; rb < n_rb; rb += gridDim.x) {
    const int tile0 = (rb * FOLD_WPB + wave) * RT;
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int nt = 0; nt < NTN; ++nt) acc[r][nt] = f32x4{0, 0, 0, 0};
    // term t sits in buffer t mod 2 and is requested one term ahead
    for (int k = 0; k < K; k += 2) {
      if (k + 1 < K) load(k + 1, b4, b1);
      compute(k, a4, a1);
      if (k + 1 < K) {
        if (k + 2 < K) load(k + 2, a4, a1);
        compute(k + 1, b4, b1);
      }
    }
    // the next block's first term (its loads overlap these stores)
    if (rb + (int)gridDim.x < n_rb) {
      rows(rb + gridDim.x);
      load(0, a4, a1);
    }
#pragma unroll
    for (int r = 0; r < RT; ++r)
#pragma unroll
      for (int nt = 0; nt < NTN; ++nt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int o = (tile0 + r) * 16 + 4 * lk + v;
          const int c = cg0 + nt * 16 + li;
          if (o < N && c < C) {
            const int q = c / 3, ch = c - 3 * q;
            B[((int64_t)q * N + perm[o]) * 3 + ch] = acc[r][nt][v];
          }
        }
  }
}

size_t folded_lds_bytes(int K, int Psh) { return sizeof(float) * (size_t)K * Psh * FOLD_LDW; }

template <int NTN, int MS>
static void folded_lds_rt(dim3 gx, int tiles, hipStream_t st, const float *P, int Psh, int K,
                          const float *Lg, int Cs, int C, int N, const int32_t *perm, float *B) {
  // Resident workgroups: as many as fit two per compute unit (LDS allowing),
  // split over the column groups; each takes row blocks of FOLD_WPB RT
  // tiles in turn.  RT = 2 unless one tile per wave fills the resident
  // slots, round by round, more than 10% better.
  const size_t lds = folded_lds_bytes(K, Psh);
  const int per_cu = std::max(1, std::min(2, (int)((160 * 1024) / lds)));
  const int gy = (int)gx.y;
  const int slots = std::max(1, 256 * per_cu / gy);
  auto fill = [&](int rt) {
    const int nrb = (tiles + FOLD_WPB * rt - 1) / (FOLD_WPB * rt);
    return (double)nrb / ((double)((nrb + slots - 1) / slots) * slots);
  };
  const int rt = fill(1) > 1.1 * fill(2) ? 1 : 2;
  const int gxx = std::min((tiles + FOLD_WPB * rt - 1) / (FOLD_WPB * rt), slots);
  if (rt == 2)
    TLT_LAUNCH((k_folded_lds<NTN, MS, 2>), dim3(gxx, gy), dim3(FOLD_WPB * 64), lds, st, P, Psh, K, Lg,
               Cs, C, N, perm, B);
  else
    TLT_LAUNCH((k_folded_lds<NTN, MS, 1>), dim3(gxx, gy), dim3(FOLD_WPB * 64), lds, st, P, Psh, K, Lg,
               Cs, C, N, perm, B);
}

template <int NTN>
static hipError_t folded_lds_ms(dim3 gx, int tiles, hipStream_t st, const float *P, int Psh, int K,
                                const float *Lg, int Cs, int C, int N, const int32_t *perm, float *B) {
  switch (Psh / 4) {
#define CASE(m) \
  case m: folded_lds_rt<NTN, m>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, perm, B); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(6) CASE(7) CASE(8) CASE(9) CASE(12) CASE(16)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipSuccess;
}

template <typename CT, int NTN, int MS>
static void folded_rt(dim3 gx, int tiles, hipStream_t st, const CT *P, int Psh, int K, const CT *Lg,
                      int Cs, int C, int N, const int32_t *perm, CT *B) {
  // tiles per wave: the most that still leaves >= 512 workgroups
  if ((tiles + 15) / 16 >= 512)
    TLT_LAUNCH((k_folded<CT, NTN, MS, 4>), dim3((tiles + 15) / 16, gx.y), dim3(256), 0, st, P, Psh, K,
               Lg, Cs, C, N, perm, B);
  else if ((tiles + 7) / 8 >= 512)
    TLT_LAUNCH((k_folded<CT, NTN, MS, 2>), dim3((tiles + 7) / 8, gx.y), dim3(256), 0, st, P, Psh, K,
               Lg, Cs, C, N, perm, B);
  else
    TLT_LAUNCH((k_folded<CT, NTN, MS, 1>), dim3((tiles + 3) / 4, gx.y), dim3(256), 0, st, P, Psh, K,
               Lg, Cs, C, N, perm, B);
}

template <typename CT, int NTN>
static hipError_t folded_ms(dim3 gx, int tiles, hipStream_t st, const CT *P, int Psh, int K,
                            const CT *Lg, int Cs, int C, int N, const int32_t *perm, CT *B) {
  switch (Psh / 4) {
#define CASE(m) \
  case m: folded_rt<CT, NTN, m>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, perm, B); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(6) CASE(7) CASE(8) CASE(9) CASE(12) CASE(16)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipSuccess;
}

template <typename CT>
static hipError_t folded_go(int C, int Cs, dim3 gx, int tiles, hipStream_t st, const CT *P, int Psh,
                            int K, const CT *Lg, int N, const int32_t *perm, CT *B) {
  // real column tiles of the widest group
  const int ntn = (std::min(FOLD_CG, C) + 15) / 16;
  switch (ntn) {
    case 1: return folded_ms<CT, 1>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, perm, B);
    case 2: return folded_ms<CT, 2>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, perm, B);
    case 3: return folded_ms<CT, 3>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, perm, B);
    default: return folded_ms<CT, 4>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, perm, B);
  }
}

size_t folded_scratch_bytes(int K, int Psh, int Cs, bool fp64) {
  return (size_t)K * Psh * Cs * (fp64 ? 8 : 4);
}

hipError_t launch_folded(const void *P, int Psh, int n_sh, int K, const void *gcol, int Cs,
                         const void *sh, Cols cols, int N, const int32_t *perm, void *B, bool fp64,
                         void *scratch, hipStream_t st) {
  if (Psh > 64 || Cs % 16 != 0) return hipErrorInvalidValue;
  const int nw = K * Psh * Cs;
  const int tiles = (N + 15) / 16;
  const dim3 gx(1, (Cs + FOLD_CG - 1) / FOLD_CG);
  hipError_t e;
  if (fp64) {
    TLT_LAUNCH(k_fold_weights<double>, dim3((nw + 255) / 256), dim3(256), 0, st,
               (const double *)gcol, Cs, (const double *)sh, cols, K, Psh, n_sh, (double *)scratch);
    e = folded_go<double>(cols.C, Cs, gx, tiles, st, (const double *)P, Psh, K,
                          (const double *)scratch, N, perm, (double *)B);
  } else {
    TLT_LAUNCH(k_fold_weights<float>, dim3((nw + 255) / 256), dim3(256), 0, st,
               (const float *)gcol, Cs, (const float *)sh, cols, K, Psh, n_sh, (float *)scratch);
    if (folded_lds_bytes(K, Psh) <= 144 * 1024) {
      const int ntn = (std::min(FOLD_CG, cols.C) + 15) / 16;
      const float *Pf = (const float *)P, *Lf = (const float *)scratch;
      switch (ntn) {
        case 1: e = folded_lds_ms<1>(gx, tiles, st, Pf, Psh, K, Lf, Cs, cols.C, N, perm, (float *)B); break;
        case 2: e = folded_lds_ms<2>(gx, tiles, st, Pf, Psh, K, Lf, Cs, cols.C, N, perm, (float *)B); break;
        case 3: e = folded_lds_ms<3>(gx, tiles, st, Pf, Psh, K, Lf, Cs, cols.C, N, perm, (float *)B); break;
        default: e = folded_lds_ms<4>(gx, tiles, st, Pf, Psh, K, Lf, Cs, cols.C, N, perm, (float *)B); break;
      }
    } else {
      e = folded_go<float>(cols.C, Cs, gx, tiles, st, (const float *)P, Psh, K, (const float *)scratch,
                           N, perm, (float *)B);
    }
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint of the transport.
//
//   gbar[k][c]  = sum_o dB[c](perm[o]) * V[k][o][c]
//   X[c][lm]    = sum_o dB[c](perm[o]) * sum_k g[k][c] P[k][o][lm]
// Per-block partial sums to scratch, then a fixed-order sum over blocks in
// float64, then thetabar = sum gbar dg and dSH from X.  The float64 path
// uses one thread per output value and block (ADJ_VB vertices).
// ---------------------------------------------------------------------------

constexpr int ADJ_VB = 256;   // vertices per block of the float64 path
constexpr int ADJ_SPLIT = 16; // first-stage groups of the block reduction

// Vertices per block of the float32 path: enough blocks to fill the chip.
static int adj_block_vertices(int N, bool fp64) {
  if (fp64) return ADJ_VB;
  int vb = 256;
  while (vb > 32 && (N + vb - 1) / vb < 1024) vb >>= 1;
  return vb;
}

// Scratch layout: per-block partials [nblk][nout] (compute type), the
// first-stage float64 sums [ADJ_SPLIT][nout], the final float64 sums [nout],
// and (float32) the Morton-ordered upstream gradient [N][Cs].
struct AdjLayout {
  size_t part, stage1, red, y, total;
};
static size_t a256(size_t x) { return (x + 255) / 256 * 256; }
static AdjLayout adj_layout(int N, int K, int n_sh, int C, int Cs, bool fp64) {
  const size_t nblk = (N + adj_block_vertices(N, fp64) - 1) / adj_block_vertices(N, fp64);
  const size_t nout = (size_t)K * C + (size_t)C * n_sh;
  AdjLayout l;
  l.part = 0;
  l.stage1 = a256(nblk * nout * (fp64 ? 8 : 4));
  l.red = l.stage1 + a256((size_t)ADJ_SPLIT * nout * 8);
  l.y = l.red + a256(nout * 8);
  l.total = l.y + (fp64 ? 0 : sizeof(float) * (size_t)N * Cs);
  return l;
}

size_t adjoint_partial_bytes(int N, int K, int n_sh, int C, int Cs, bool fp64) {
  return adj_layout(N, K, n_sh, C, Cs, fp64).total;
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

// float32 storage: the same partial sums from three streaming kernels.
//   k_adj_permute: Y[o][c] = dB[c](perm[o]) in Morton order (stride Cs);
//   k_adj_gbar:    gbar partials, V and Y streamed as float4 rows (all K
//                  terms of a vertex block per workgroup, Y rows staged in
//                  LDS once, when they fit);
//   k_adj_x:       X partials as a matrix product on the matrix cores over
//                  the contraction index kappa = (k, o):
//                  X[c][lm] += sum_kappa (g[k][c] Y[o][c]) * P[k][o][lm],
//                  v_mfma_f32_16x16x4f32 (exact float32 products, float32
//                  accumulation).

__global__ __launch_bounds__(256) void k_adj_permute(const float *__restrict__ dB,
                                                     const int32_t *__restrict__ perm, int N, int C,
                                                     int Cs, float *__restrict__ Y) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= (int64_t)N * Cs) return;
  const int o = (int)(i / Cs), c = (int)(i - (int64_t)o * Cs);
  float y = 0.f;
  if (c < C) {
    const int q = c / 3, ch = c - 3 * q;
    y = dB[((int64_t)q * N + perm[o]) * 3 + ch];
  }
  Y[i] = y;
}

// All K terms of a vertex block in one workgroup: the block's Y rows are
// staged in LDS once (grid nblk; Y read once instead of once per term).
__global__ __launch_bounds__(256) void k_adj_gbar_all(const float *__restrict__ V,
                                                      const float *__restrict__ Y, int Cs, int N,
                                                      int C, int K, int nout, int vb,
                                                      float *__restrict__ part) {
  extern __shared__ float4 ys[];     // [vb][Cs/4]
  __shared__ float4 red[256];
  const int t = threadIdx.x;
  const int b = blockIdx.x;
  const int o0 = b * vb;
  const int nv = min(vb, N - o0);
  const int cq = Cs / 4;
  const int R = 256 / cq;
  const int q4 = t % cq, r = t / cq;
  const float4 *y4 = reinterpret_cast<const float4 *>(Y + (int64_t)o0 * Cs);
  for (int i = t; i < nv * cq; i += 256) ys[i] = y4[i];
  __syncthreads();
  for (int k = 0; k < K; ++k) {
    float4 acc = {0.f, 0.f, 0.f, 0.f};
    if (r < R) {
      const float4 *v4 = reinterpret_cast<const float4 *>(V + ((int64_t)k * N + o0) * Cs) + q4;
#pragma unroll 4
      for (int ol = r; ol < nv; ol += R) {
        const float4 v = v4[(int64_t)ol * cq];
        const float4 y = ys[ol * cq + q4];
        acc.x = fmaf(v.x, y.x, acc.x);
        acc.y = fmaf(v.y, y.y, acc.y);
        acc.z = fmaf(v.z, y.z, acc.z);
        acc.w = fmaf(v.w, y.w, acc.w);
      }
    }
    red[t] = acc;
    __syncthreads();
    if (t < cq) {
      float4 s = red[t];
      for (int rr = 1; rr < R; ++rr) {
        const float4 x = red[rr * cq + t];
        s.x += x.x;
        s.y += x.y;
        s.z += x.z;
        s.w += x.w;
      }
      const float sv[4] = {s.x, s.y, s.z, s.w};
      for (int u = 0; u < 4; ++u) {
        const int c = 4 * t + u;
        if (c < C) part[(size_t)b * nout + (size_t)k * C + c] = sv[u];
      }
    }
    __syncthreads();
  }
}

// grid (nblk, K): block b, term k.  Thread = (row phase r, column quad).
__global__ __launch_bounds__(256) void k_adj_gbar(const float *__restrict__ V,
                                                  const float *__restrict__ Y, int Cs, int N, int C,
                                                  int nout, int vb, float *__restrict__ part) {
  __shared__ float4 red[256];
  const int t = threadIdx.x;
  const int b = blockIdx.x, k = blockIdx.y;
  const int o0 = b * vb;
  const int nv = min(vb, N - o0);
  const int cq = Cs / 4;            // column quads (Cs is a multiple of 16)
  const int R = 256 / cq;           // rows in flight per pass
  const int q4 = t % cq, r = t / cq;
  float4 acc = {0.f, 0.f, 0.f, 0.f};
  if (r < R) {
    const float4 *v4 = reinterpret_cast<const float4 *>(V + ((int64_t)k * N + o0) * Cs) + q4;
    const float4 *y4 = reinterpret_cast<const float4 *>(Y + (int64_t)o0 * Cs) + q4;
#pragma unroll 4
    for (int ol = r; ol < nv; ol += R) {
      const float4 v = v4[(int64_t)ol * cq];
      const float4 y = y4[(int64_t)ol * cq];
      acc.x = fmaf(v.x, y.x, acc.x);
      acc.y = fmaf(v.y, y.y, acc.y);
      acc.z = fmaf(v.z, y.z, acc.z);
      acc.w = fmaf(v.w, y.w, acc.w);
    }
  }
  red[t] = acc;
  __syncthreads();
  if (t < cq) {
    float4 s = red[t];
    for (int rr = 1; rr < R; ++rr) {
      const float4 x = red[rr * cq + t];
      s.x += x.x;
      s.y += x.y;
      s.z += x.z;
      s.w += x.w;
    }
    const float sv[4] = {s.x, s.y, s.z, s.w};
    for (int u = 0; u < 4; ++u) {
      const int c = 4 * t + u;
      if (c < C) part[(size_t)b * nout + (size_t)k * C + c] = sv[u];
    }
  }
}

// X partials of block b and column group blockIdx.y (64 columns): every wave
// takes a quarter of the block's vertices, four at a time, and for each term
// k multiplies A = (g_k[c] Y[o][c]) by B = P_k[o][lm] into its (c, lm) tiles
// (MTN x NTN tiles of 16x16 in registers).  Loads carry no branches:
// addresses are clamped, values past the ends zeroed.  The four waves'
// tiles are then added in wave order through LDS.
template <int MTN, int NTN, int KT>
__global__ __launch_bounds__(256) void k_adj_x(const float *__restrict__ Y, int Cs,
                                               const float *__restrict__ P, int Psh,
                                               const float *__restrict__ gcol, int N, int K,
                                               int n_sh, int C, int nout, int vb,
                                               float *__restrict__ part) {
  __shared__ float red[64 * 64];
  __shared__ float gl[16 * 64];   // K <= 16
  const int t = threadIdx.x;
  const int wave = t >> 6, lane = t & 63, li = lane & 15, lk = lane >> 4;
  const int b = blockIdx.x, cg0 = blockIdx.y * 64;
  const int n_g = K * C;
  for (int i = t; i < K * 64; i += 256) {
    const int c = cg0 + (i & 63);
    gl[i] = c < C ? gcol[(size_t)(i >> 6) * Cs + c] : 0.f;
  }
  __syncthreads();
  const int per = vb / 4;
  const int ow0 = b * vb + wave * per;
  const int ow1 = min(ow0 + per, N);
  f32x4 acc[MTN][NTN];
#pragma unroll
  for (int m = 0; m < MTN; ++m)
#pragma unroll
    for (int n = 0; n < NTN; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
  int ycol[MTN];
#pragma unroll
  for (int m = 0; m < MTN; ++m) ycol[m] = min(cg0 + m * 16 + li, Cs - 1);
  int pcol[NTN];
  bool pok[NTN];
#pragma unroll
  for (int n = 0; n < NTN; ++n) {
    pok[n] = n * 16 + li < n_sh;
    pcol[n] = min(n * 16 + li, Psh - 1);
  }
  for (int o = ow0; o < ow1; o += 4) {
    const int orow = o + lk;
    const bool ook = orow < ow1;
    const int oc = min(orow, N - 1);
    float yv[MTN];
#pragma unroll
    for (int m = 0; m < MTN; ++m) yv[m] = Y[(int64_t)oc * Cs + ycol[m]];
    float pv[KT][NTN];   // KT >= K; rows past K repeat row K-1 and are not used
#pragma unroll
    for (int k = 0; k < KT; ++k)
#pragma unroll
      for (int n = 0; n < NTN; ++n) pv[k][n] = P[((int64_t)min(k, K - 1) * N + oc) * Psh + pcol[n]];
#pragma unroll
    for (int m = 0; m < MTN; ++m) yv[m] = ook ? yv[m] : 0.f;
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (k < K) {
#pragma unroll
        for (int m = 0; m < MTN; ++m) {
          const float a = gl[k * 64 + m * 16 + li] * yv[m];
#pragma unroll
          for (int n = 0; n < NTN; ++n)
            acc[m][n] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, pok[n] ? pv[k][n] : 0.f, acc[m][n], 0, 0, 0);
        }
      }
    }
  }
  // the four waves' tiles, added in wave order
  for (int w = 0; w < 4; ++w) {
    if (wave == w) {
#pragma unroll
      for (int m = 0; m < MTN; ++m)
#pragma unroll
        for (int n = 0; n < NTN; ++n)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int idx = (m * 16 + 4 * lk + v) * 64 + n * 16 + li;
            red[idx] = (w == 0 ? 0.f : red[idx]) + acc[m][n][v];
          }
    }
    __syncthreads();
  }
  for (int i = t; i < 64 * 64; i += 256) {
    const int cl = i >> 6, lm = i & 63, c = cg0 + cl;
    if (c < C && lm < n_sh) part[(size_t)b * nout + n_g + (size_t)c * n_sh + lm] = red[i];
  }
}

template <int MTN, int KT>
static void adj_x_go(int ntn, dim3 g, hipStream_t st, const float *Y, int Cs, const float *P, int Psh,
                     const float *gcol, int N, int K, int n_sh, int C, int nout, int vb, float *part) {
  switch (ntn) {
#define ADJX(n)                                                                                 \
  case n:                                                                                       \
    TLT_LAUNCH((k_adj_x<MTN, n, KT>), g, dim3(256), 0, st, Y, Cs, P, Psh, gcol, N, K, n_sh, C, \
               nout, vb, part);                                                                 \
    break;
    ADJX(1) ADJX(2) ADJX(3) ADJX(4)
#undef ADJX
  }
}

template <int MTN>
static void adj_x_k(int ntn, dim3 g, hipStream_t st, const float *Y, int Cs, const float *P, int Psh,
                    const float *gcol, int N, int K, int n_sh, int C, int nout, int vb, float *part) {
  if (K <= 4) adj_x_go<MTN, 4>(ntn, g, st, Y, Cs, P, Psh, gcol, N, K, n_sh, C, nout, vb, part);
  else if (K <= 8) adj_x_go<MTN, 8>(ntn, g, st, Y, Cs, P, Psh, gcol, N, K, n_sh, C, nout, vb, part);
  else adj_x_go<MTN, 16>(ntn, g, st, Y, Cs, P, Psh, gcol, N, K, n_sh, C, nout, vb, part);
}

// Sum of the per-block partials in a fixed order, in float64.  Stage 1:
// grid (output chunks of 64, ADJ_SPLIT groups of blocks); lane = output,
// wave w sums a contiguous quarter of the group's blocks, the quarters are
// added in order.  Stage 2: the ADJ_SPLIT group sums, in order.
template <typename CT>
__global__ __launch_bounds__(256) void k_adj_reduce(const CT *__restrict__ part, int nblk, int nout,
                                                    double *__restrict__ stage1) {
  __shared__ double q4[4][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int t = blockIdx.x * 64 + lane;
  const int g = blockIdx.y;
  const int g0 = (int)((int64_t)nblk * g / ADJ_SPLIT), g1 = (int)((int64_t)nblk * (g + 1) / ADJ_SPLIT);
  const int b0 = g0 + (int)((int64_t)(g1 - g0) * w / 4), b1 = g0 + (int)((int64_t)(g1 - g0) * (w + 1) / 4);
  double s = 0.0;
  if (t < nout) {
#pragma unroll 4
    for (int bb = b0; bb < b1; ++bb) s += (double)part[(size_t)bb * nout + t];
  }
  q4[w][lane] = s;
  __syncthreads();
  if (w == 0 && t < nout)
    stage1[(size_t)g * nout + t] = ((q4[0][lane] + q4[1][lane]) + q4[2][lane]) + q4[3][lane];
}

__global__ __launch_bounds__(256) void k_adj_reduce2(const double *__restrict__ stage1, int nout,
                                                     double *__restrict__ out) {
  const int t = blockIdx.x * 256 + threadIdx.x;
  if (t >= nout) return;
  double s = 0.0;
  for (int g = 0; g < ADJ_SPLIT; ++g) s += stage1[(size_t)g * nout + t];
  out[t] = s;
}

// thetabar[m][ch][p] and dSH[l][lm][ch] from the reduced sums.
template <typename CT>
__global__ void k_adj_out(const double *__restrict__ red, const double *__restrict__ dg64, int K,
                          int n_sh, Cols cols, CT *__restrict__ dSH, double *__restrict__ dTheta) {
  const int gt = blockIdx.x * blockDim.x + threadIdx.x;
  const int C = cols.C;
  const double *gbar = red;             // [K][C]
  const double *X = red + (size_t)K * C; // [C][n_sh]
  const int n_th = cols.n_mat * 9;
  const int n_l = cols.n_light * n_sh * 3;
  if (gt < n_th * 64) {
    // one wave per material derivative: lanes take (output set, term)
    // pairs with independent loads, then a fixed-order wave sum
    const int t = gt >> 6, lane = gt & 63;
    const int m = t / 9, ch = (t / 3) % 3, p = t % 3;
    double s = 0.0;
    for (int i = lane; i < cols.n_out * K; i += 64) {
      const int q = i / K, k = i - q * K;
      const int mq = cols.n_mat > 1 ? q : 0;
      if (mq == m) s += gbar[(size_t)k * C + 3 * q + ch] * dg64[(((size_t)m * 3 + ch) * K + k) * 3 + p];
    }
    s = wave_sum(s);
    if (lane == 0) dTheta[t] = s;
  } else if (gt < n_th * 64 + n_l) {
    const int u = gt - n_th * 64;
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
  const int vb = adj_block_vertices(N, fp64);
  const int nblk = (N + vb - 1) / vb;
  const int nout = K * C + C * n_sh;
  const AdjLayout l = adj_layout(N, K, n_sh, C, Cs, fp64);
  if (partial_bytes < l.total) return hipErrorInvalidValue;
  double *stage1 = (double *)((char *)partial + l.stage1);
  double *red = (double *)((char *)partial + l.red);
  const int n_fin = cols.n_mat * 9 * 64 + cols.n_light * n_sh * 3;  // a wave per material derivative
  const dim3 gr((nout + 63) / 64, ADJ_SPLIT);
  if (fp64) {
    const dim3 g1(nblk, (nout + 255) / 256);
    TLT_LAUNCH(k_adj_partial<double>, g1, dim3(256), 0, st, (const double *)dB,
                       (const double *)V, Cs, (const double *)P, Psh, (const double *)gcol, perm,
                       N, K, n_sh, C, (double *)partial);
    TLT_LAUNCH(k_adj_reduce<double>, gr, dim3(256), 0, st, (const double *)partial, nblk,
                       nout, stage1);
  } else {
    if (Cs % 16 != 0 || Cs > 1024 || Psh > 64 || K > 16 || n_sh > 64) return hipErrorInvalidValue;
    float *Y = (float *)((char *)partial + l.y);
    const int64_t ny = (int64_t)N * Cs;
    // (a vertex-major form with scattered row writes measured 2.6x slower)
    TLT_LAUNCH(k_adj_permute, dim3((unsigned)((ny + 255) / 256)), dim3(256), 0, st,
               (const float *)dB, perm, N, C, Cs, Y);
    // one workgroup per block for all terms when there are enough blocks to
    // fill the chip and the block's Y rows fit the LDS budget
    const size_t ylds = sizeof(float) * (size_t)vb * Cs;
    if (ylds <= 64 * 1024 && nblk >= 1024)
      TLT_LAUNCH(k_adj_gbar_all, dim3(nblk), dim3(256), ylds, st, (const float *)V, Y, Cs, N, C, K,
                 nout, vb, (float *)partial);
    else
      TLT_LAUNCH(k_adj_gbar, dim3(nblk, K), dim3(256), 0, st, (const float *)V, Y, Cs, N, C,
                 nout, vb, (float *)partial);
    {
      const dim3 gx(nblk, (C + 63) / 64);
      const int mtn = (std::min(64, C) + 15) / 16, ntn = (n_sh + 15) / 16;
      const float *Pf = (const float *)P, *gf = (const float *)gcol;
      float *pf = (float *)partial;
      if (mtn == 1) adj_x_k<1>(ntn, gx, st, Y, Cs, Pf, Psh, gf, N, K, n_sh, C, nout, vb, pf);
      else if (mtn == 2) adj_x_k<2>(ntn, gx, st, Y, Cs, Pf, Psh, gf, N, K, n_sh, C, nout, vb, pf);
      else if (mtn == 3) adj_x_k<3>(ntn, gx, st, Y, Cs, Pf, Psh, gf, N, K, n_sh, C, nout, vb, pf);
      else adj_x_k<4>(ntn, gx, st, Y, Cs, Pf, Psh, gf, N, K, n_sh, C, nout, vb, pf);
    }
    TLT_LAUNCH(k_adj_reduce<float>, gr, dim3(256), 0, st, (const float *)partial, nblk,
                       nout, stage1);
  }
  TLT_LAUNCH(k_adj_reduce2, dim3((nout + 255) / 256), dim3(256), 0, st, stage1, nout, red);
  if (fp64)
    TLT_LAUNCH(k_adj_out<double>, dim3((n_fin + 255) / 256), dim3(256), 0, st, red, dg64,
                       K, n_sh, cols, (double *)dSH, dTheta);
  else
    TLT_LAUNCH(k_adj_out<float>, dim3((n_fin + 255) / 256), dim3(256), 0, st, red, dg64,
                       K, n_sh, cols, (float *)dSH, dTheta);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Read-bandwidth probe (measurement only): every workgroup streams its
// share of a buffer with 16-byte buffer loads, sixteen in flight per lane,
// and folds the words into one value it writes out (so the loads are not
// dropped).  Reads past the end return zeros.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_read_probe(const void *__restrict__ buf, int64_t bytes,
                                                    uint32_t *__restrict__ out) {
  const int64_t per = (bytes + gridDim.x - 1) / gridDim.x;
  const int64_t begin = (per + 4095) / 4096 * 4096 * blockIdx.x;
  const int64_t end = min(bytes, begin + (per + 4095) / 4096 * 4096);
  uint32_t acc = 0;
  if (begin < end) {
    const int64_t len = end - begin;
    const __amdgpu_buffer_rsrc_t r = __builtin_amdgcn_make_buffer_rsrc(
        (void *)((const char *)buf + begin), (short)0, (int)min<int64_t>(len, 0x7fffffff), 0x00020000);
    for (int64_t off = 0; off < len; off += 16 * 256 * 16) {
      uint4 v[16];
#pragma unroll
      for (int u = 0; u < 16; ++u)
        v[u] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                             r, (int)(off + (u * 256 + threadIdx.x) * 16), 0, 0));
#pragma unroll
      for (int u = 0; u < 16; ++u) acc ^= v[u].x + v[u].y + v[u].z + v[u].w;
    }
  }
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) out[blockIdx.x * 4 + (threadIdx.x >> 6)] = acc;
}

hipError_t launch_read_probe(const void *buf, int64_t bytes, uint32_t *out, int blocks, hipStream_t st) {
  if (blocks < 1 || bytes < 0 || (bytes + blocks - 1) / blocks > 0x70000000) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_read_probe, dim3(blocks), dim3(256), 0, st, buf, bytes, out);
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
