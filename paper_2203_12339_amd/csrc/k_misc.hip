// Small kernels: material-only combine, adjoint reductions, storage
// conversion at load time.

#include "device_common.h"

namespace tlt {

// Material-only update (Steps 3-4 of Sec. 4): B = sum_k g_k v_k from the
// v_k kept by the last full render, [N][K][Cs] with vertices in original
// order (so the output rows are written where they are read).  One thread per (vertex,
// column).
template <typename CT>
__global__ __launch_bounds__(256) void k_combine(const CT *__restrict__ V, int Cs,
                                                 const CT *__restrict__ gcol, int K, int N, int C,
                                                 CT *__restrict__ B) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)N * C) return;
  const int v = (int)(t / C), c = (int)(t - (int64_t)v * C);
  CT s = 0;
  for (int k = 0; k < K; ++k) s = fma(gcol[(size_t)k * Cs + c], V[((int64_t)v * K + k) * Cs + c], s);
  const int q = c / 3, ch = c - 3 * q;
  B[((int64_t)q * N + v) * 3 + ch] = s;
}

// Float32 form over tiles of CMB_V vertices x CMB_W columns (16 output
// sets; Cs is a multiple of 16 and CMB_W of 3 and 16): every thread takes
// CMB_Q column quads of the tile and issues the 16-byte loads of all KT <= 16
// terms before the sums; the sums go to LDS, and the tile's rows of each
// output set are then written as one contiguous run of 3 * CMB_V floats.
constexpr int CMB_V = 64, CMB_W = 48, CMB_Q = CMB_V * (CMB_W / 4) / 256;

template <int KT>
__global__ __launch_bounds__(256) void k_combine4(const float *__restrict__ V, int Cs,
                                                  const float *__restrict__ gcol, int K, int N, int C,
                                                  float *__restrict__ B) {
  __shared__ float bs[CMB_W][CMB_V + 1];
  const int t = threadIdx.x;
  const int v0 = blockIdx.x * CMB_V, cg0 = blockIdx.y * CMB_W;
  float4 v[CMB_Q][KT];
#pragma unroll
  for (int i = 0; i < CMB_Q; ++i) {
    const int item = t + 256 * i;                 // (vertex, quad) of the tile
    const int vl = item / (CMB_W / 4), c0 = cg0 + 4 * (item % (CMB_W / 4));
    const int vtx = min(v0 + vl, N - 1), cc = min(c0, Cs - 4);
#pragma unroll
    for (int k = 0; k < KT; ++k)
      v[i][k] = *reinterpret_cast<const float4 *>(V + ((int64_t)vtx * K + min(k, K - 1)) * Cs + cc);
  }
#pragma unroll
  for (int i = 0; i < CMB_Q; ++i) {
    const int item = t + 256 * i;
    const int vl = item / (CMB_W / 4), ql = item % (CMB_W / 4), c0 = cg0 + 4 * ql;
    const int cc = min(c0, Cs - 4);
    float s[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int k = 0; k < KT; ++k) {
      if (k < K) {
        const float4 g = *reinterpret_cast<const float4 *>(gcol + (size_t)k * Cs + cc);
        s[0] = fmaf(g.x, v[i][k].x, s[0]);
        s[1] = fmaf(g.y, v[i][k].y, s[1]);
        s[2] = fmaf(g.z, v[i][k].z, s[2]);
        s[3] = fmaf(g.w, v[i][k].w, s[3]);
      }
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) bs[4 * ql + j][vl] = s[j];
  }
  __syncthreads();
  // set q of the tile: B[q][v0 .. v0 + CMB_V)[0..2], contiguous
  const int nv = min(CMB_V, N - v0);
  for (int i = t; i < (CMB_W / 3) * 3 * CMB_V; i += 256) {
    const int ql = i / (3 * CMB_V), r = i - ql * 3 * CMB_V;
    const int vl = r / 3, ch = r - 3 * vl;
    const int c = cg0 + 3 * ql + ch;
    if (vl < nv && c < C) B[((int64_t)(c / 3) * N + v0) * 3 + r] = bs[3 * ql + ch][vl];
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

hipError_t launch_combine(const void *V, int Cs, const void *gcol, int K, int N, int C, void *B,
                          bool fp64, hipStream_t st) {
  const int64_t n = (int64_t)N * C;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (fp64)
    TLT_LAUNCH(k_combine<double>, dim3(blocks), dim3(256), 0, st, (const double *)V, Cs,
               (const double *)gcol, K, N, C, (double *)B);
  else if (Cs % 16 == 0 && K <= 16) {
    const dim3 g((N + CMB_V - 1) / CMB_V, (C + CMB_W - 1) / CMB_W);
    const float *Vf = (const float *)V, *gf = (const float *)gcol;
    if (K <= 4)
      TLT_LAUNCH(k_combine4<4>, g, dim3(256), 0, st, Vf, Cs, gf, K, N, C, (float *)B);
    else if (K <= 8)
      TLT_LAUNCH(k_combine4<8>, g, dim3(256), 0, st, Vf, Cs, gf, K, N, C, (float *)B);
    else
      TLT_LAUNCH(k_combine4<16>, g, dim3(256), 0, st, Vf, Cs, gf, K, N, C, (float *)B);
  } else
    TLT_LAUNCH(k_combine<float>, dim3(blocks), dim3(256), 0, st, (const float *)V, Cs,
               (const float *)gcol, K, N, C, (float *)B);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Folded lighting transport (Eq. 14, the SH lighting path): with
// P_k = W_k H (A o T) (built at load, [N][K][Psh] with vertices in original
// order, so row o of the product is output vertex o),
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
    prow[r] = P + (int64_t)min(o, N - 1) * K * Psh;
  }
  int bcol[NTN];
#pragma unroll
  for (int nt = 0; nt < NTN; ++nt) bcol[nt] = min(cg0 + nt * 16 + li, Cs - 1);
  for (int k = 0; k < K; ++k) {
    const int64_t koff = (int64_t)k * Psh;
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
          B[((int64_t)q * N + o) * 3 + ch] = acc[r][nt][v];
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
    const int64_t koff = (int64_t)k * Psh;
#pragma unroll
    for (int r = 0; r < RT; ++r) {
#pragma unroll
      for (int g = 0; g < G4; ++g)
        x4[r][g] = *reinterpret_cast<const float4 *>(prow[r] + koff + idx::fold_group_index(g, lk, 0));
#pragma unroll
      for (int q = 0; q < R4; ++q) x1[r][q] = prow[r][koff + idx::fold_tail_index(G4, q, lk)];
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
        for (int nt = 0; nt < NTN; ++nt)
          bv[4 * g + v][nt] = lk_rows[idx::fold_group_index(g, lk, v) * FOLD_LDW + nt * 16];
#pragma unroll
    for (int q = 0; q < R4; ++q)
#pragma unroll
      for (int nt = 0; nt < NTN; ++nt)
        bv[4 * G4 + q][nt] = lk_rows[idx::fold_tail_index(G4, q, lk) * FOLD_LDW + nt * 16];
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
      prow[r] = P + (int64_t)min(o, N - 1) * K * Psh;
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
            B[((int64_t)q * N + o) * 3 + ch] = acc[r][nt][v];
          }
        }
  }
}

size_t folded_lds_bytes(int K, int Psh) { return sizeof(float) * (size_t)K * Psh * FOLD_LDW; }

template <int NTN, int MS>
static void folded_lds_rt(dim3 gx, int tiles, hipStream_t st, const float *P, int Psh, int K,
                          const float *Lg, int Cs, int C, int N, float *B) {
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
               Cs, C, N, B);
  else
    TLT_LAUNCH((k_folded_lds<NTN, MS, 1>), dim3(gxx, gy), dim3(FOLD_WPB * 64), lds, st, P, Psh, K, Lg,
               Cs, C, N, B);
}

template <int NTN>
static hipError_t folded_lds_ms(dim3 gx, int tiles, hipStream_t st, const float *P, int Psh, int K,
                                const float *Lg, int Cs, int C, int N, float *B) {
  switch (Psh / 4) {
#define CASE(m) \
  case m: folded_lds_rt<NTN, m>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, B); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(6) CASE(7) CASE(8) CASE(9) CASE(12) CASE(16)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipSuccess;
}

template <typename CT, int NTN, int MS>
static void folded_rt(dim3 gx, int tiles, hipStream_t st, const CT *P, int Psh, int K, const CT *Lg,
                      int Cs, int C, int N, CT *B) {
  // tiles per wave: the most that still leaves >= 512 workgroups
  if ((tiles + 15) / 16 >= 512)
    TLT_LAUNCH((k_folded<CT, NTN, MS, 4>), dim3((tiles + 15) / 16, gx.y), dim3(256), 0, st, P, Psh, K,
               Lg, Cs, C, N, B);
  else if ((tiles + 7) / 8 >= 512)
    TLT_LAUNCH((k_folded<CT, NTN, MS, 2>), dim3((tiles + 7) / 8, gx.y), dim3(256), 0, st, P, Psh, K,
               Lg, Cs, C, N, B);
  else
    TLT_LAUNCH((k_folded<CT, NTN, MS, 1>), dim3((tiles + 3) / 4, gx.y), dim3(256), 0, st, P, Psh, K,
               Lg, Cs, C, N, B);
}

template <typename CT, int NTN>
static hipError_t folded_ms(dim3 gx, int tiles, hipStream_t st, const CT *P, int Psh, int K,
                            const CT *Lg, int Cs, int C, int N, CT *B) {
  switch (Psh / 4) {
#define CASE(m) \
  case m: folded_rt<CT, NTN, m>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, B); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(6) CASE(7) CASE(8) CASE(9) CASE(12) CASE(16)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipSuccess;
}

template <typename CT>
static hipError_t folded_go(int C, int Cs, dim3 gx, int tiles, hipStream_t st, const CT *P, int Psh,
                            int K, const CT *Lg, int N, CT *B) {
  // real column tiles of the widest group
  const int ntn = (std::min(FOLD_CG, C) + 15) / 16;
  switch (ntn) {
    case 1: return folded_ms<CT, 1>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, B);
    case 2: return folded_ms<CT, 2>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, B);
    case 3: return folded_ms<CT, 3>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, B);
    default: return folded_ms<CT, 4>(gx, tiles, st, P, Psh, K, Lg, Cs, C, N, B);
  }
}

static size_t fold16_scratch(int K, int Psh, int Cs);

size_t folded_scratch_bytes(int K, int Psh, int Cs, bool fp64) {
  const size_t lg = (size_t)K * Psh * Cs * (fp64 ? 8 : 4);
  return fp64 ? lg : std::max(lg, fold16_scratch(K, Psh, Cs));
}

// ---------------------------------------------------------------------------
// Folded lighting on an FP16 copy of P (16-bit transport storage).  At load
// P [N][K][Psh] (float32) is scaled by a power of two sp, which puts its
// largest magnitude in [2^13, 2^14), and written in the A-operand fragment
// order of v_mfma_f32_16x16x32_f16: fragment (16-row tile t, step s) holds
// for lane l the eight values P[16 t + l % 16][32 s + 8 (l / 16) + i],
// i = 0..7, over the contraction index j = k Psh + lm (zero past N and past
// J = K Psh), so a wave reads one contiguous 1 KB per step.  Per frame the
// weighted lighting Lg[(k, lm)][c] = g_k[c] L[lm][c] is written once as
// B-operand fragments per 64-column group (k_fold_lg16, straight from g_k
// and L): each column scaled by a power of two (from a bound on its largest
// magnitude, so nothing exceeds the FP16 range) and split into FP16 hi + lo,
// so Lg keeps about 22 significant bits; each workgroup copies its group's
// fragments into LDS.  B = P Lg then runs on
// the FP16 matrix instructions with float32 accumulation, and the epilogue
// undoes both scales (exactly: powers of two).  The P stream is half of the
// float32 form's and the matrix work a small fraction of its time.
// ---------------------------------------------------------------------------

typedef _Float16 h16x8 __attribute__((ext_vector_type(8)));

// Largest |P| as float bits (non-negative floats order as unsigned ints;
// a value that is not finite reports +inf).
__global__ __launch_bounds__(256) void k_fold_absmax(const float *__restrict__ P, int64_t n,
                                                     unsigned *__restrict__ out) {
  float m = 0.f;
  for (int64_t i = blockIdx.x * 256LL + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    const float v = fabsf(P[i]);
    m = (v <= 3.0e38f) ? fmaxf(m, v) : __builtin_inff();
  }
  for (int off = 32; off > 0; off >>= 1) m = fmaxf(m, __shfl_xor(m, off, 64));
  if ((threadIdx.x & 63) == 0) atomicMax(out, __float_as_uint(m));
}

// One lane slot (16 bytes) of the FP16 copy per thread.
__global__ __launch_bounds__(256) void k_fold_pack(const float *__restrict__ P, int N, int J, int S,
                                                   float sp, h16x8 *__restrict__ P16) {
  const int64_t f = blockIdx.x * 256LL + threadIdx.x;
  if (f >= (int64_t)((N + 15) / 16) * S * 64) return;
  const int l = (int)(f & 63);
  const int64_t ts = f >> 6;
  const int s = (int)(ts % S);
  const int64_t o = (ts / S) * 16 + (l & 15);
  const int j0 = 32 * s + 8 * (l >> 4);
  h16x8 v;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int j = j0 + i;
    v[i] = (o < N && j < J) ? (_Float16)(P[o * J + j] * sp) : (_Float16)0.f;
  }
  P16[f] = v;
}

constexpr int F16_WPB = 8;   // waves per workgroup (one 16-row tile each per round)

// Weighted lighting as FP16 B-operand fragments, per 64-column group y:
// lgf[y][s][nt][h][l] holds for lane slot l the eight values
// Lg[32 s + 8 (l / 16) + i][c] (c = 64 y + 16 nt + l % 16, Lg[(k, lm)][c] =
// g_k[c] L[light(c)][lm][ch(c)]) times the column scale csc[c], split hi
// (h = 0) and lo (h = 1).  csc[c] is the power of two that puts the bound
// max_k |g_k[c]| max_lm |L[light(c)][lm][ch(c)]| in [2^13, 2^14), so no
// scaled value exceeds the FP16 range.  One thread per lane slot.
__global__ __launch_bounds__(256) void k_fold_lg16(const float *__restrict__ gcol, int Cs,
                                                   const float *__restrict__ sh, Cols cols, int K,
                                                   int Psh, int n_sh, int S, int NTN, int gy,
                                                   h16x8 *__restrict__ lgf, float *__restrict__ cscg) {
  const int f = blockIdx.x * 256 + threadIdx.x;
  const int per_group = S * NTN * 64;
  if (f >= gy * per_group) return;
  const int y = f / per_group, r = f - y * per_group;
  const int l = r & 63, snt = r >> 6;
  const int cl = (snt % NTN) * 16 + (l & 15), c = y * 64 + cl;
  const int j0 = 32 * (snt / NTN) + 8 * (l >> 4);
  const int J = K * Psh;
  float sc = 1.f;
  float v[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) v[i] = 0.f;
  if (c < cols.C) {
    const int q = c / 3, ch = c - 3 * q;
    const float *L = sh + (size_t)(cols.n_light > 1 ? q : 0) * n_sh * 3 + ch;
    float mg = 0.f, mL = 0.f;
#pragma unroll 8
    for (int k = 0; k < K; ++k) mg = fmaxf(mg, fabsf(gcol[(size_t)k * Cs + c]));
#pragma unroll 12
    for (int lm = 0; lm < n_sh; ++lm) mL = fmaxf(mL, fabsf(L[lm * 3]));
    const float bound = mg * mL;
    int e = 0;
    (void)frexpf(bound, &e);
    sc = bound > 0.f ? ldexpf(1.f, 14 - e) : 1.f;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int j = j0 + i, k = j / Psh, lm = j - k * Psh;
      if (j < J && lm < n_sh) v[i] = gcol[(size_t)k * Cs + c] * L[lm * 3] * sc;
    }
  }
  h16x8 hi, lo;
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const _Float16 h = (_Float16)v[i];
    hi[i] = h;
    lo[i] = (_Float16)(v[i] - (float)h);
  }
  lgf[(size_t)(y * S * NTN + snt) * 128 + l] = hi;
  lgf[(size_t)(y * S * NTN + snt) * 128 + 64 + l] = lo;
  if (snt < NTN && l < 16) cscg[y * 64 + cl] = sc;   // step 0, lane group 0: one thread per column
}

// S steps of 32 contraction indices, NTN real 16-column tiles of the group.
// Workgroups stay resident (two per compute unit) and take rounds of
// F16_WPB tiles in turn; a wave requests the fragments of its next tile
// before the matrix work of the current one (clamped to the last tile, so
// the requests carry no branch).
template <int S, int NTN>
__global__ __launch_bounds__(F16_WPB * 64) __attribute__((amdgpu_waves_per_eu(S <= 9 ? 4 : 1))) void k_folded16(
    const h16x8 *__restrict__ P16, const h16x8 *__restrict__ lgf, const float *__restrict__ cscg, int C,
    int N, float inv_sp, float *__restrict__ B) {
  extern __shared__ __align__(16) unsigned char smem[];
  h16x8 *lf = reinterpret_cast<h16x8 *>(smem);                            // [S][NTN][2][64]
  float *csc = reinterpret_cast<float *>(smem + (size_t)S * NTN * 2 * 64 * 16);  // [64]
  const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
  const int cg0 = blockIdx.y * FOLD_CG;
  const int tiles = (N + 15) / 16;
  const int n_rounds = (tiles + F16_WPB - 1) / F16_WPB;
  const int G = gridDim.x;
  auto load = [&](int rb, h16x8 (&dst)[S]) {
    const int tile = min(rb * F16_WPB + wave, tiles - 1);
    const h16x8 *src = P16 + (int64_t)tile * S * 64 + lane;
#pragma unroll
    for (int s = 0; s < S; ++s) dst[s] = src[s * 64];
  };
  // the first tile's fragments are requested before the staging
  h16x8 a0[S], a1[S];
  load(blockIdx.x, a0);
  // the group's lighting fragments and column scales (k_fold_lg16) into LDS:
  // every load issued before the stores
  {
    constexpr int NSL = S * NTN * 2 * 64, PER = (NSL + F16_WPB * 64 - 1) / (F16_WPB * 64);
    const h16x8 *src = lgf + (size_t)blockIdx.y * NSL;
    h16x8 v[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) v[u] = src[min(u * F16_WPB * 64 + t, NSL - 1)];
#pragma unroll
    for (int u = 0; u < PER; ++u)
      if (u * F16_WPB * 64 + t < NSL) lf[u * F16_WPB * 64 + t] = v[u];
    if (t < 64) csc[t] = cscg[blockIdx.y * 64 + t];
  }
  __syncthreads();
  float inv_c[NTN];
#pragma unroll
  for (int nt = 0; nt < NTN; ++nt) inv_c[nt] = inv_sp / csc[nt * 16 + (lane & 15)];
  auto compute = [&](int rb, const h16x8 (&a)[S]) {
    // the staged fragments are the same for every tile: without this fence
    // the compiler keeps all of them in registers (S NTN 8 VGPRs) instead of
    // reading each from LDS next to its matrix instruction
    __asm__ volatile("" ::: "memory");
    f32x4 acc[NTN];
#pragma unroll
    for (int nt = 0; nt < NTN; ++nt) acc[nt] = f32x4{0, 0, 0, 0};
#pragma unroll
    for (int s = 0; s < S; ++s)
#pragma unroll
      for (int nt = 0; nt < NTN; ++nt)
#pragma unroll
        for (int h = 0; h < 2; ++h)
          acc[nt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[s], lf[((s * NTN + nt) * 2 + h) * 64 + lane],
                                                            acc[nt], 0, 0, 0);
    const int tile = rb * F16_WPB + wave;
#pragma unroll
    for (int nt = 0; nt < NTN; ++nt)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int o = tile * 16 + 4 * (lane >> 4) + v;
        const int c = cg0 + nt * 16 + (lane & 15);
        if (o < N && c < C) {
          const int q = c / 3, ch = c - 3 * q;
          B[((int64_t)q * N + o) * 3 + ch] = acc[nt][v] * inv_c[nt];
        }
      }
  };
  for (int rb = blockIdx.x; rb < n_rounds; rb += 2 * G) {
    load(rb + G, a1);
    compute(rb, a0);
    if (rb + G >= n_rounds) break;
    load(rb + 2 * G, a0);
    compute(rb + G, a1);
  }
}

size_t fold16_bytes(int N, int J) {
  const int S = (J + 31) / 32;
  return (size_t)((N + 15) / 16) * S * 64 * 16;
}

hipError_t launch_fold_absmax(const float *P, int64_t n, unsigned *absmax, hipStream_t st) {
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 4096);
  TLT_LAUNCH(k_fold_absmax, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, st, P, n, absmax);
  return hipGetLastError();
}

hipError_t launch_fold_pack(const float *P, int N, int J, float sp, void *P16, hipStream_t st) {
  const int S = (J + 31) / 32;
  if (S < 1 || S > FOLD16_MAX_STEPS) return hipErrorInvalidValue;
  const int64_t slots = (int64_t)((N + 15) / 16) * S * 64;
  TLT_LAUNCH(k_fold_pack, dim3((unsigned)((slots + 255) / 256)), dim3(256), 0, st, P, N, J, S, sp,
             (h16x8 *)P16);
  return hipGetLastError();
}

template <int S, int NTN>
static hipError_t folded16_go(const void *P16, const h16x8 *lgf, const float *cscg, int Cs, int C,
                              int N, float inv_sp, float *B, hipStream_t st) {
  const size_t lds = (size_t)S * NTN * 2 * 64 * 16 + 64 * sizeof(float);
  const int gy = (Cs + FOLD_CG - 1) / FOLD_CG;
  const int tiles = (N + 15) / 16;
  const int n_rounds = (tiles + F16_WPB - 1) / F16_WPB;
  const int per_cu = std::max(1, std::min(2, (int)((160 * 1024) / lds)));
  const int gx = std::max(1, std::min(n_rounds, 256 * per_cu / gy));
  TLT_LAUNCH((k_folded16<S, NTN>), dim3(gx, gy), dim3(F16_WPB * 64), lds, st, (const h16x8 *)P16, lgf,
             cscg, C, N, inv_sp, B);
  return hipGetLastError();
}

template <int S>
static hipError_t folded16_nt(int ntn, const void *P16, const h16x8 *lgf, const float *cscg, int Cs,
                              int C, int N, float inv_sp, float *B, hipStream_t st) {
  switch (ntn) {
    case 1: return folded16_go<S, 1>(P16, lgf, cscg, Cs, C, N, inv_sp, B, st);
    case 2: return folded16_go<S, 2>(P16, lgf, cscg, Cs, C, N, inv_sp, B, st);
    case 3: return folded16_go<S, 3>(P16, lgf, cscg, Cs, C, N, inv_sp, B, st);
    default: return folded16_go<S, 4>(P16, lgf, cscg, Cs, C, N, inv_sp, B, st);
  }
}

// scratch of the FP16 form: fragments [gy][S][NTN][2][64] (16 bytes each,
// NTN = 4 at most) and column scales [gy][64]
static size_t fold16_scratch(int K, int Psh, int Cs) {
  const int S = (K * Psh + 31) / 32, gy = (Cs + FOLD_CG - 1) / FOLD_CG;
  return (size_t)gy * S * 4 * 128 * 16 + (size_t)gy * 64 * sizeof(float);
}

static hipError_t launch_folded16(const void *P16, const float *gcol, const float *sh, Cols cols,
                                  int K, int Psh, int n_sh, int Cs, int N, float inv_sp, float *B,
                                  void *scratch, hipStream_t st) {
  const int C = cols.C, J = K * Psh, S = (J + 31) / 32;
  const int ntn = (std::min(FOLD_CG, C) + 15) / 16;
  const int gy = (Cs + FOLD_CG - 1) / FOLD_CG;
  if (S < 1 || S > FOLD16_MAX_STEPS) return hipErrorInvalidValue;
  h16x8 *lgf = (h16x8 *)scratch;
  float *cscg = (float *)((char *)scratch + (size_t)gy * S * 4 * 128 * 16);
  const int slots = gy * S * ntn * 64;
  TLT_LAUNCH(k_fold_lg16, dim3((slots + 255) / 256), dim3(256), 0, st, gcol, Cs, sh, cols, K, Psh, n_sh,
             S, ntn, gy, lgf, cscg);
  switch (S) {
#define F16S(s) case s: return folded16_nt<s>(ntn, P16, lgf, cscg, Cs, C, N, inv_sp, B, st);
    F16S(1) F16S(2) F16S(3) F16S(4) F16S(5) F16S(6) F16S(7) F16S(8)
    F16S(9) F16S(10) F16S(11) F16S(12) F16S(13) F16S(14) F16S(15) F16S(16)
#undef F16S
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_folded(const void *P, int Psh, int n_sh, int K, const void *gcol, int Cs,
                         const void *sh, Cols cols, int N, void *B, bool fp64,
                         void *scratch, hipStream_t st, const void *P16, float p16_inv) {
  if (Psh > 64 || Cs % 16 != 0) return hipErrorInvalidValue;
  const int nw = K * Psh * Cs;
  const int tiles = (N + 15) / 16;
  const dim3 gx(1, (Cs + FOLD_CG - 1) / FOLD_CG);
  hipError_t e;
  if (P16 != nullptr) {
    if (fp64) return hipErrorInvalidValue;
    e = launch_folded16(P16, (const float *)gcol, (const float *)sh, cols, K, Psh, n_sh, Cs, N, p16_inv,
                        (float *)B, scratch, st);
  } else if (fp64) {
    TLT_LAUNCH(k_fold_weights<double>, dim3((nw + 255) / 256), dim3(256), 0, st,
               (const double *)gcol, Cs, (const double *)sh, cols, K, Psh, n_sh, (double *)scratch);
    e = folded_go<double>(cols.C, Cs, gx, tiles, st, (const double *)P, Psh, K,
                          (const double *)scratch, N, (double *)B);
  } else {
    TLT_LAUNCH(k_fold_weights<float>, dim3((nw + 255) / 256), dim3(256), 0, st,
               (const float *)gcol, Cs, (const float *)sh, cols, K, Psh, n_sh, (float *)scratch);
    if (folded_lds_bytes(K, Psh) <= 144 * 1024) {
      const int ntn = (std::min(FOLD_CG, cols.C) + 15) / 16;
      const float *Pf = (const float *)P, *Lf = (const float *)scratch;
      switch (ntn) {
        case 1: e = folded_lds_ms<1>(gx, tiles, st, Pf, Psh, K, Lf, Cs, cols.C, N, (float *)B); break;
        case 2: e = folded_lds_ms<2>(gx, tiles, st, Pf, Psh, K, Lf, Cs, cols.C, N, (float *)B); break;
        case 3: e = folded_lds_ms<3>(gx, tiles, st, Pf, Psh, K, Lf, Cs, cols.C, N, (float *)B); break;
        default: e = folded_lds_ms<4>(gx, tiles, st, Pf, Psh, K, Lf, Cs, cols.C, N, (float *)B); break;
      }
    } else {
      e = folded_go<float>(cols.C, Cs, gx, tiles, st, (const float *)P, Psh, K, (const float *)scratch,
                           N, (float *)B);
    }
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Adjoint of the transport.  Steps 1-4 of Sec. 4 are linear in the lighting
// and in the weights g_k, and with the lighting-transfer product
// P_k = W_k H pad(A o T) (built at load, [N][K][Psh] with vertices in original
// order) the per-term transport is v_k = P_k L.  Both gradients therefore follow from
//   Z_k[lm][c] = sum_v P_k[v][lm] dB[q][v][ch]          (c = 3 q + ch)
//   gbar[k][c] = sum_lm L[light(q)][lm][ch] Z_k[lm][c]   (d loss / d g_k)
//   X[c][lm]   = sum_k g_k[c] Z_k[lm][c]                 (d loss / d L)
// P and the upstream gradient dB are each read once, contiguously.  Partial
// sums of gbar and X per workgroup go to scratch, then a fixed-order float64
// sum over the partial rows, then thetabar = sum gbar dg/dtheta and dSH
// from X.
// ---------------------------------------------------------------------------

constexpr int ADJ_VB = 256;   // vertices per partial row of the float64 path
constexpr int ADJ_SPLIT = 16; // first-stage groups of the row reduction

// float32 path (k_adj_z): one wave per term, eight terms per workgroup,
// output sets in groups of 16 (48 columns), the upstream gradient staged in
// LDS in blocks of 64 vertices (column-major, AZ_YS floats per column),
// vertex ranges split into about AZ_TARGET workgroups (two per compute unit)
// in steps of 4 vertices.
constexpr int AZ_VB = 64, AZ_W = 48, AZ_YS = 68, AZ_WAVES = 8, AZ_TARGET = 512, AZ_PD = 8;

struct AdjGeom {
  int nrow;     // partial rows
  int nwg;      // vertex ranges
  int nz;       // term groups (float32 path)
  int ngroups;  // column groups (float32 path)
  int span;     // vertices per range
};

static AdjGeom adj_geom(int N, int K, int C, bool fp64) {
  AdjGeom g;
  if (fp64) {
    g.nwg = (N + ADJ_VB - 1) / ADJ_VB;
    g.nz = g.ngroups = 1;
    g.span = ADJ_VB;
    g.nrow = g.nwg;
    return g;
  }
  g.ngroups = (C + AZ_W - 1) / AZ_W;
  g.nz = (K + AZ_WAVES - 1) / AZ_WAVES;
  const int want = std::max(1, AZ_TARGET / (g.ngroups * g.nz));
  g.span = std::max(4, ((N + want - 1) / want + 3) / 4 * 4);
  g.nwg = (N + g.span - 1) / g.span;
  g.nrow = g.nwg * g.nz;
  return g;
}

// Scratch layout: partial rows [nrow][nout] (compute type) and the
// first-stage float64 sums [ADJ_SPLIT][nout].
struct AdjLayout {
  size_t part, stage1, total;
};
static size_t a256(size_t x) { return (x + 255) / 256 * 256; }
static AdjLayout adj_layout(int N, int K, int n_sh, int C, bool fp64) {
  const AdjGeom g = adj_geom(N, K, C, fp64);
  const size_t nout = (size_t)K * C + (size_t)C * n_sh;
  AdjLayout l;
  l.part = 0;
  l.stage1 = a256((size_t)g.nrow * nout * (fp64 ? 8 : 4));
  l.total = l.stage1 + a256((size_t)ADJ_SPLIT * nout * 8);
  return l;
}

size_t adjoint_partial_bytes(int N, int K, int n_sh, int C, bool fp64) {
  return adj_layout(N, K, n_sh, C, fp64).total;
}

// float64 path: one thread per output value and partial row (ADJ_VB
// vertices).
template <typename CT>
__global__ __launch_bounds__(256) void k_adj_partial(const CT *__restrict__ dB,
                                                     const CT *__restrict__ P, int Psh,
                                                     const CT *__restrict__ gcol, int Cs,
                                                     const CT *__restrict__ sh, Cols cols, int N,
                                                     int K, int n_sh, CT *__restrict__ part) {
  const int t = blockIdx.y * 256 + threadIdx.x;
  const int C = cols.C;
  const int n_g = K * C, n_x = C * n_sh;
  if (t >= n_g + n_x) return;
  const int v0 = blockIdx.x * ADJ_VB;
  const int v1 = min(N, v0 + ADJ_VB);
  CT acc = 0;
  if (t < n_g) {
    const int k = t / C, c = t - k * C;
    const int q = c / 3, ch = c - 3 * q;
    const CT *Lc = sh + (size_t)(cols.n_light > 1 ? q : 0) * n_sh * 3 + ch;
    for (int v = v0; v < v1; ++v) {
      const CT *pr = P + ((int64_t)v * K + k) * Psh;
      CT pl = 0;
      for (int lm = 0; lm < n_sh; ++lm) pl = fma(pr[lm], Lc[3 * lm], pl);
      acc = fma(dB[((int64_t)q * N + v) * 3 + ch], pl, acc);
    }
  } else {
    const int u = t - n_g;
    const int c = u / n_sh, lm = u - c * n_sh;
    const int q = c / 3, ch = c - 3 * q;
    for (int v = v0; v < v1; ++v) {
      CT s = 0;
      for (int k = 0; k < K; ++k) s = fma(gcol[(size_t)k * Cs + c], P[((int64_t)v * K + k) * Psh + lm], s);
      acc = fma(dB[((int64_t)q * N + v) * 3 + ch], s, acc);
    }
  }
  part[(size_t)blockIdx.x * (n_g + n_x) + t] = acc;
}

// float32 path.  Grid (vertex ranges, column groups, term groups); wave w
// of term group z owns term k = 8 z + w and accumulates Z_k of its column
// group over its range on the matrix cores, v_mfma_f32_16x16x4_f32 (exact
// float32 products, float32 accumulation) with
//   A[i][kk] = dB at (vertex 4 s + kk, column 16 ct + i)   (staged in LDS)
//   B[kk][j] = P_k[vertex 4 s + kk][NL j + u]              (from HBM)
// so tile (ct, u) of lane (j, lg) holds Z_k[NL j + u][16 ct + 4 lg + v] in
// component v.  Each lane loads NL consecutive P values per step (the 16
// lanes of a vertex cover a whole P row), through a register ring PD steps
// ahead of use that runs across the staged blocks.  The gradient block of
// the next 64 vertices is loaded during the current block's matrix work:
// lane l of a wave takes vertex l of two output sets (three contiguous
// channels each, 768 contiguous bytes per wave and set).  In the
// column-major staging (stride AZ_YS = 68) both the staging stores (64
// vertices of one column) and the A-operand reads (16 columns x 4 vertices)
// of a wave fall on 64 distinct banks.
template <int NCT, int NL>
__global__ __launch_bounds__(AZ_WAVES * 64) __attribute__((amdgpu_waves_per_eu(4))) void k_adj_z(const float *__restrict__ dB,
                                                         const float *__restrict__ P, int Psh,
                                                         const float *__restrict__ gcol, int Cs,
                                                         const float *__restrict__ sh, Cols cols,
                                                         int N, int K, int n_sh, int span, int nout,
                                                         float *__restrict__ part) {
  __shared__ __align__(16) float ys[2][AZ_W * AZ_YS];   // [column][vertex], vertices >= 64 unused
  __shared__ float xs[AZ_W * 64];                        // [column][lm]
  __shared__ float ls[AZ_W * 64];                        // L of the group's columns, [column][lm]
  __shared__ float gs[AZ_WAVES * AZ_W];                  // g_k of the group's terms and columns
  constexpr int NTHR = AZ_WAVES * 64;
  constexpr int GI = AZ_W * AZ_VB / NTHR;                // staged values per thread
  // the wave index is uniform: read it as such, so the term's buffer
  // resource and branches are scalar
  const int t = threadIdx.x, wave = __builtin_amdgcn_readfirstlane(t >> 6);
  const int lane = t & 63, li = lane & 15, lg = lane >> 4;
  const int C = cols.C;
  const int cg0 = blockIdx.y * AZ_W;
  const int cw = min(AZ_W, C - cg0);   // real columns of the group (a multiple of 3)
  const int q0 = cg0 / 3, nq = cw / 3;
  const int z = blockIdx.z;
  const int k = z * AZ_WAVES + wave;
  const bool active = k < K;
  const int v_begin = blockIdx.x * span;
  const int v_end = min(N, v_begin + span);
  const int nv = v_end - v_begin;
  const int nblk = (nv + AZ_VB - 1) / AZ_VB;
  const int64_t row = (int64_t)blockIdx.x * gridDim.z + z;

  // Thread t stages vertex t % 64 of output sets t / 64 and t / 64 + 8 (three
  // channels each).
  static_assert(NTHR == 8 * 64 && GI == 6, "staging map: 8 waves x 64 vertices x 2 sets x 3 channels");
  const int vl_t = t & 63, qa = wave, qb = qa + 8;
  const bool qa_ok = qa < nq, qb_ok = qb < nq;
  const float *gsa = dB + ((int64_t)(q0 + (qa_ok ? qa : 0)) * N + v_begin + vl_t) * 3;
  const float *gsb = dB + ((int64_t)(q0 + (qb_ok ? qb : 0)) * N + v_begin + vl_t) * 3;
  // L and g_k of the group, for the epilogue, staged once (zeros past the
  // group's columns and n_sh)
  for (int i = t; i < AZ_W * 64; i += NTHR) {
    const int cl = i >> 6, lm = i & 63, c = cg0 + cl;
    float x = 0.f;
    if (cl < cw && lm < n_sh) {
      const int q = c / 3, ch = c - 3 * q;
      x = sh[((size_t)(cols.n_light > 1 ? q : 0) * n_sh + lm) * 3 + ch];
    }
    ls[i] = x;
  }
  for (int i = t; i < AZ_WAVES * AZ_W; i += NTHR) {
    const int kk = z * AZ_WAVES + i / AZ_W, cl = i % AZ_W;
    gs[i] = (kk < K && cl < cw) ? gcol[(size_t)kk * Cs + cg0 + cl] : 0.f;
  }

  float gv[GI];
  // Branch-free: the loads always run (the vertex clamped into range) and
  // values outside the range or the group are zeroed only when stored, so no
  // load sits under a branch and nothing waits on the gather before the
  // block's matrix work -- the P ring's wait counts stay exact.
  auto gather = [&](int blk) {
    const int v = min(v_begin + blk * AZ_VB + vl_t, N - 1);
    const int64_t off = (int64_t)(v - v_begin - vl_t) * 3;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      gv[ch] = gsa[off + ch];
      gv[3 + ch] = gsb[off + ch];
    }
  };
  // every (column, vertex) slot of the buffer is written, zeros outside the
  // range and the group's real columns
  auto stage = [&](int buf, int blk) {
    const bool v_ok = v_begin + blk * AZ_VB + vl_t < v_end;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
      ys[buf][(3 * qa + ch) * AZ_YS + vl_t] = (qa_ok && v_ok) ? gv[ch] : 0.f;
      ys[buf][(3 * qb + ch) * AZ_YS + vl_t] = (qb_ok && v_ok) ? gv[3 + ch] : 0.f;
    }
  };

  // The range's P rows (all K terms of a vertex are contiguous, so the
  // workgroup's waves read one stream) through a buffer resource: a step's
  // lane offset is one 32-bit add, and reads past the range return zeros.
  const bool lok = NL * li < Psh;
  const __amdgpu_buffer_rsrc_t prs = __builtin_amdgcn_make_buffer_rsrc(
      (void *)(P + (int64_t)v_begin * K * Psh), (short)0, nv * K * Psh * (int)sizeof(float),
      0x00020000);
  const int step_b = 4 * K * Psh * (int)sizeof(float);
  const int lane_b = ((lg * K + min(k, K - 1)) * Psh + (lok ? NL * li : 0)) * (int)sizeof(float);
  auto load_p = [&](int sg, float (&dst)[NL]) {
    const int off = lane_b + sg * step_b;
#pragma unroll
    for (int u = 0; u < NL; ++u)
      dst[u] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(prs, off + 4 * u, 0, 0));
  };

  f32x4 acc[NCT][NL];
#pragma unroll
  for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
    for (int u = 0; u < NL; ++u) acc[ct][u] = f32x4{0.f, 0.f, 0.f, 0.f};
  float ring[AZ_PD][NL];
#pragma unroll
  for (int p = 0; p < AZ_PD; ++p) load_p(p, ring[p]);

  gather(0);
  stage(0, 0);
  __syncthreads();
  for (int blk = 0; blk < nblk; ++blk) {
    const int buf = blk & 1;
    gather(blk + 1);   // past the last block: clamped, never stored
    // the gathered values are stored to LDS after this block's matrix work:
    // keep the scheduler from pulling the stores (and their wait on the
    // gather, which would drain the P ring) up here
    __builtin_amdgcn_sched_barrier(0);
    const int ns = min(AZ_VB / 4, (nv - blk * AZ_VB + 3) / 4);   // steps of this block
    const float *yb = ys[buf] + li * AZ_YS + lg;
    // Every block runs all its steps' ring refills (straight-line code, so
    // the wait counts are the same on every path); steps past the range only
    // skip their matrix work (their P reads return zeros past the range).
#pragma unroll
    for (int g0 = 0; g0 < AZ_VB / 4; g0 += AZ_PD) {
#pragma unroll
      for (int p = 0; p < AZ_PD; ++p) {
        const int s = g0 + p;
        if (active && s < ns) {
          float av[NCT];
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) av[ct] = yb[16 * ct * AZ_YS + 4 * s];
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
            for (int u = 0; u < NL; ++u)
              acc[ct][u] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[ct], lok ? ring[p][u] : 0.f,
                                                                acc[ct][u], 0, 0, 0);
        }
        load_p(blk * (AZ_VB / 4) + s + AZ_PD, ring[p]);  // refill PD steps ahead
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    if (blk + 1 < nblk) stage(buf ^ 1, blk + 1);
    __syncthreads();
  }

  // gbar partials of this wave's term: sum over lm within the lane's
  // column, then over the 16 lanes of a lane group
  if (active) {
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int cl = 16 * ct + 4 * lg + v, c = cg0 + cl;
        float sg = 0.f;
#pragma unroll
        for (int u = 0; u < NL; ++u) sg = fmaf(ls[cl * 64 + NL * li + u], acc[ct][u][v], sg);
        sg += __shfl_xor(sg, 1, 64);
        sg += __shfl_xor(sg, 2, 64);
        sg += __shfl_xor(sg, 4, 64);
        sg += __shfl_xor(sg, 8, 64);
        if (li == 0 && c < cg0 + cw) part[row * nout + (int64_t)k * C + c] = sg;
      }
  }
  // terms of other term groups are zero in this row
  for (int i = t; i < K * cw; i += NTHR) {
    const int kk = i / cw, c = cg0 + i % cw;
    if (kk / AZ_WAVES != z) part[row * nout + (int64_t)kk * C + c] = 0.f;
  }
  // X partials: g_k-weighted Z_k of the waves, added in wave order
  for (int w = 0; w < AZ_WAVES; ++w) {
    if (wave == w && active) {
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int cl = 16 * ct + 4 * lg + v;
          const float gk = gs[wave * AZ_W + cl];
#pragma unroll
          for (int u = 0; u < NL; ++u) {
            const int idx = cl * 64 + NL * li + u;
            xs[idx] = (w == 0 ? 0.f : xs[idx]) + gk * acc[ct][u][v];
          }
        }
    }
    __syncthreads();
  }
  for (int i = t; i < cw * n_sh; i += NTHR) {
    const int cl = i / n_sh, lm = i - cl * n_sh;
    part[row * nout + (int64_t)K * C + (int64_t)(cg0 + cl) * n_sh + lm] = xs[cl * 64 + lm];
  }
}

template <int NCT>
static hipError_t adj_z_nl(int nl, dim3 g, hipStream_t st, const float *dB, const float *P, int Psh,
                           const float *gcol, int Cs, const float *sh, Cols cols, int N, int K,
                           int n_sh, int span, int nout, float *part) {
  switch (nl) {
#define AZ(n)                                                                                      \
  case n:                                                                                          \
    TLT_LAUNCH((k_adj_z<NCT, n>), g, dim3(AZ_WAVES * 64), 0, st, dB, P, Psh, gcol, Cs, sh, cols, N, \
               K, n_sh, span, nout, part);                                                         \
    return hipSuccess;
    AZ(1) AZ(2) AZ(3) AZ(4)
#undef AZ
  }
  return hipErrorInvalidValue;
}

// Sum of the partial rows in a fixed order, in float64.  Stage 1: grid
// (output chunks of 64, ADJ_SPLIT groups of rows); lane = output, wave w sums
// a contiguous quarter of the group's rows, the quarters are added in order.
// Stage 2 (in k_adj_final): the ADJ_SPLIT group sums, in order.
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

// thetabar[m][ch][p] and dSH[l][lm][ch] straight from the ADJ_SPLIT group
// sums: every reduced value is the sum of its groups in order (as a second
// reduction pass would form it), taken where it is used.
template <typename CT>
__global__ __launch_bounds__(256) void k_adj_final(const double *__restrict__ stage1, int nout,
                                                   const double *__restrict__ dg64, int K, int n_sh,
                                                   Cols cols, CT *__restrict__ dSH,
                                                   double *__restrict__ dTheta) {
  const int gt = blockIdx.x * 256 + threadIdx.x;
  const int C = cols.C;
  const int n_th = cols.n_mat * 9;
  auto red = [&](size_t i) {
    double s = 0.0;
#pragma unroll
    for (int g = 0; g < ADJ_SPLIT; ++g) s += stage1[(size_t)g * nout + i];
    return s;
  };
  if (gt < n_th * 64) {
    // one wave per material derivative: lanes take (output set, term) pairs
    // with independent loads, then a fixed-order wave sum
    const int d = gt >> 6, lane = gt & 63;
    const int m = d / 9, ch = (d / 3) % 3, p = d % 3;
    double s = 0.0;
    for (int i = lane; i < cols.n_out * K; i += 64) {
      const int q = i / K, k = i - q * K;
      const int mq = cols.n_mat > 1 ? q : 0;
      if (mq == m) s += red((size_t)k * C + 3 * q + ch) * dg64[(((size_t)m * 3 + ch) * K + k) * 3 + p];
    }
    s = wave_sum(s);
    if (lane == 0) dTheta[d] = s;
  } else if (gt < n_th * 64 + cols.n_light * n_sh * 3) {
    const int u = gt - n_th * 64;
    const int l = u / (n_sh * 3), lm = (u / 3) % n_sh, ch = u % 3;
    double s = 0.0;
    for (int q = 0; q < cols.n_out; ++q) {
      const int lq = cols.n_light > 1 ? q : 0;
      if (lq == l) s += red((size_t)K * C + (size_t)(3 * q + ch) * n_sh + lm);
    }
    dSH[u] = (CT)s;
  }
}

hipError_t launch_adjoint(const void *dB, const void *P, int Psh, const void *gcol, int Cs,
                          const void *sh, const double *dg64, int N, int K, int n_sh, Cols cols,
                          bool fp64, void *partial, size_t partial_bytes, void *dSH, double *dTheta,
                          hipStream_t st) {
  const int C = cols.C;
  const int nout = K * C + C * n_sh;
  const AdjGeom geo = adj_geom(N, K, C, fp64);
  const AdjLayout l = adj_layout(N, K, n_sh, C, fp64);
  if (partial_bytes < l.total) return hipErrorInvalidValue;
  double *stage1 = (double *)((char *)partial + l.stage1);
  const dim3 gr((nout + 63) / 64, ADJ_SPLIT);
  if (fp64) {
    const dim3 g1(geo.nwg, (nout + 255) / 256);
    TLT_LAUNCH(k_adj_partial<double>, g1, dim3(256), 0, st, (const double *)dB, (const double *)P, Psh,
               (const double *)gcol, Cs, (const double *)sh, cols, N, K, n_sh, (double *)partial);
    TLT_LAUNCH(k_adj_reduce<double>, gr, dim3(256), 0, st, (const double *)partial, geo.nrow, nout,
               stage1);
  } else {
    if (Psh > 64 || n_sh > Psh || Psh % ((Psh + 15) / 16) != 0) return hipErrorInvalidValue;
    const dim3 gz(geo.nwg, geo.ngroups, geo.nz);
    const int nct = (std::min(AZ_W, C) + 15) / 16, nl = (Psh + 15) / 16;
    const float *dBf = (const float *)dB, *Pf = (const float *)P, *gf = (const float *)gcol;
    const float *shf = (const float *)sh;
    float *pf = (float *)partial;
    hipError_t e;
    if (nct == 1) e = adj_z_nl<1>(nl, gz, st, dBf, Pf, Psh, gf, Cs, shf, cols, N, K, n_sh, geo.span, nout, pf);
    else if (nct == 2) e = adj_z_nl<2>(nl, gz, st, dBf, Pf, Psh, gf, Cs, shf, cols, N, K, n_sh, geo.span, nout, pf);
    else e = adj_z_nl<3>(nl, gz, st, dBf, Pf, Psh, gf, Cs, shf, cols, N, K, n_sh, geo.span, nout, pf);
    if (e != hipSuccess) return e;
    TLT_LAUNCH(k_adj_reduce<float>, gr, dim3(256), 0, st, (const float *)partial, geo.nrow, nout, stage1);
  }
  const int n_fin = cols.n_mat * 9 * 64 + cols.n_light * n_sh * 3;  // a wave per material derivative
  if (fp64)
    TLT_LAUNCH(k_adj_final<double>, dim3((n_fin + 255) / 256), dim3(256), 0, st, stage1, nout, dg64, K,
               n_sh, cols, (double *)dSH, dTheta);
  else
    TLT_LAUNCH(k_adj_final<float>, dim3((n_fin + 255) / 256), dim3(256), 0, st, stage1, nout, dg64, K,
               n_sh, cols, (float *)dSH, dTheta);
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
