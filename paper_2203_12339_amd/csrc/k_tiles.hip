// a4 + a5 on block-dense tiles: the wavelet-sparse transport of Eq. (7)/(8)
// (rendering Steps 2 and 4 of Sec. 4) as 16x16 matrix-instruction tiles.
//
// A block holds the R = V*K rows (o, k) of V Morton-consecutive vertices,
// dense over the sorted union U of their kept columns (about half of the
// slots are kept coefficients, the rest zeros).  One workgroup per block
// (and 16*NT-column group), one wave per 16-row m-tile:
//
//   D[row, c] = sum_u W[row, u] * Ehat[U[u], c]       (MFMA, FP32 accumulate)
//   B[o, c]   = sum_k g_k[c] * D[(o,k), c]            (K-term fusion)
//
// W streams from HBM once, in fragment order (one contiguous 256 B or 1 KB
// load per wave and step).  The gathered irradiance rows Ehat[U[u]] are
// read once per block into LDS, already in B-operand fragment order, and
// shared by every wave -- each gathered row serves all V*K rows of the
// block.  With 16-bit storage Ehat is split into hi + lo 16-bit parts (two
// instructions per tile), so the product keeps ~16 significant bits of
// Ehat; W itself is exact in the instruction's input type.
//
// Kinds: 0 = f32 storage, v_mfma_f32_16x16x4_f32 (exact FP32 products);
//        1 = bf16 storage, v_mfma_f32_16x16x32_bf16 with bf16 hi/lo Ehat;
//        2 = f16 storage,  v_mfma_f32_16x16x32_f16 with f16 hi/lo Ehat.
// Operand layout (measured on gfx950): lane l supplies A[l%16][kpl*(l/16)+i]
// and B[kpl*(l/16)+i][l%16], i < kpl; result v of lane l is D[4*(l/16)+v][l%16].

#include "device_common.h"

namespace tlt {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <int KIND> struct TileKind;
template <> struct TileKind<0> {
  static constexpr int KSTEP = 4, KPL = 1, H = 1;
  typedef float AFrag;
  typedef float BFrag;
  typedef float BElem;
  static __device__ __forceinline__ f32x4 mma(AFrag a, BFrag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ AFrag load_a(const void *p, int64_t frag_elem) {
    return ((const float *)p)[frag_elem];
  }
  static __device__ __forceinline__ void split(float x, BElem &hi, BElem &lo) { hi = x; lo = 0; }
};
template <> struct TileKind<1> {
  static constexpr int KSTEP = 32, KPL = 8, H = 2;
  typedef bf16x8 AFrag;
  typedef bf16x8 BFrag;
  typedef __bf16 BElem;
  static __device__ __forceinline__ f32x4 mma(AFrag a, BFrag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ AFrag load_a(const void *p, int64_t frag_elem) {
    const uint4 u = *(const uint4 *)((const uint16_t *)p + frag_elem);
    return __builtin_bit_cast(AFrag, u);
  }
  static __device__ __forceinline__ void split(float x, BElem &hi, BElem &lo) {
    hi = (__bf16)x;
    lo = (__bf16)(x - (float)hi);
  }
};
template <> struct TileKind<2> {
  static constexpr int KSTEP = 32, KPL = 8, H = 2;
  typedef f16x8 AFrag;
  typedef f16x8 BFrag;
  typedef _Float16 BElem;
  static __device__ __forceinline__ f32x4 mma(AFrag a, BFrag b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ AFrag load_a(const void *p, int64_t frag_elem) {
    const uint4 u = *(const uint4 *)((const uint16_t *)p + frag_elem);
    return __builtin_bit_cast(AFrag, u);
  }
  static __device__ __forceinline__ void split(float x, BElem &hi, BElem &lo) {
    hi = (_Float16)x;
    lo = (_Float16)(x - (float)hi);
  }
};

// Work split: a workgroup owns one block and one group of NT <= 3 16-column
// tiles (wider launches run as several column groups; they re-read the same
// W block, which the XCD's L2 serves).  Its WM = MT/MTW waves each compute
// MTW m-tiles x NT n-tiles.  Per chunk of KC k-steps the gathered
// irradiance is staged once in LDS (B-operand fragment order) and read by
// every wave; each wave loads the W fragments of its own m-tiles for the
// NEXT chunk while it multiplies the current one, so the HBM latency hides
// behind a whole chunk of matrix work.
constexpr int TILE_IPT = 4;          // staged items per thread and chunk
constexpr int TILE_LDS = 32 * 1024;  // staging budget per workgroup

template <int KIND, int MTW, int NT, int KCMAX>
__global__ __launch_bounds__(512) void k_tiles(TileArgs a) {
  typedef TileKind<KIND> TK;
  typedef typename TK::BElem BElem;
  typedef typename TK::BFrag BFrag;
  typedef typename TK::AFrag AFrag;
  constexpr int KS = TK::KSTEP, KPL = TK::KPL, H = TK::H;
  constexpr int FRAG = 64 * KPL;  // elements per fragment
  extern __shared__ __align__(16) unsigned char smem[];
  BElem *stage = reinterpret_cast<BElem *>(smem);

  const int b = xcd_remap(blockIdx.x, a.n_blocks);
  if (b >= a.n_blocks) return;
  const int MT = a.R / 16;
  const int WN = a.wn;
  const int NTB = WN * NT;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int wm = wave / WN, wn = wave % WN;
  const int nthr = blockDim.x;
  const int cbase = blockIdx.y * NTB * 16;  // first column of the block's group
  const int KC = a.kc;                      // k-steps per staged chunk
  const int64_t u0 = a.blk_off[b];
  const int n_steps = (int)((a.blk_off[b + 1] - u0) / KS);
  const int n_chunks = (n_steps + KC - 1) / KC;
  const int32_t *__restrict__ ucol = a.ucol + u0;
  const float *__restrict__ ehat = (const float *)a.ehat;
  const int64_t vbase = u0 * a.R;  // first value element of this block
  const int items = KC * 4 * NTB * 16;

  // staging item = (step sl, lane group lg, column n): KPL consecutive union
  // entries of one column -> one 16-byte (or 4-byte) LDS store.
  float gat[TILE_IPT][KPL];
  auto gather = [&](int chunk) {
#pragma unroll
    for (int it = 0; it < TILE_IPT; ++it) {
      const int item = threadIdx.x + it * nthr;
      const int n = item % (NTB * 16);
      const int lg = (item / (NTB * 16)) % 4;
      const int sl = item / (NTB * 16 * 4);
      const int s = chunk * KC + sl;
      const int c = cbase + n;
      const bool ok = item < items && s < n_steps && c < a.Cs;
#pragma unroll
      for (int i = 0; i < KPL; ++i) {
        const int j = ok ? ucol[s * KS + KPL * lg + i] : 0;
        const float x = ehat[(int64_t)j * a.Cs + (ok ? c : 0)];
        gat[it][i] = ok ? x : 0.f;
      }
    }
  };
  auto stage_write = [&]() {
#pragma unroll
    for (int it = 0; it < TILE_IPT; ++it) {
      const int item = threadIdx.x + it * nthr;
      if (item < items) {
        const int n = item % (NTB * 16);
        const int lg = (item / (NTB * 16)) % 4;
        const int sl = item / (NTB * 16 * 4);
        const int nt = n / 16, ln = lg * 16 + (n % 16);
        BFrag hi, lo;
#pragma unroll
        for (int i = 0; i < KPL; ++i) {
          BElem h_, l_;
          TK::split(gat[it][i], h_, l_);
          if constexpr (KPL == 1) {
            hi = h_;
            lo = l_;
          } else {
            hi[i] = h_;
            lo[i] = l_;
          }
        }
        *reinterpret_cast<BFrag *>(stage + ((size_t)((sl * NTB + nt) * H + 0) * 64 + ln) * KPL) = hi;
        if constexpr (H == 2)
          *reinterpret_cast<BFrag *>(stage + ((size_t)((sl * NTB + nt) * H + 1) * 64 + ln) * KPL) = lo;
      }
    }
  };

  f32x4 acc[MTW][NT];
#pragma unroll
  for (int m = 0; m < MTW; ++m)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[m][nt] = f32x4{0, 0, 0, 0};

  // W fragments of a whole chunk, for this wave's m-tiles (clamped loads
  // past the last step are never used)
  auto load_a = [&](int chunk, AFrag (&dst)[KCMAX][MTW]) {
#pragma unroll
    for (int sl = 0; sl < KCMAX; ++sl) {
      const int ss = min(chunk * KC + min(sl, KC - 1), n_steps - 1);
#pragma unroll
      for (int m = 0; m < MTW; ++m) {
        const int t = wm * MTW + m;
        dst[sl][m] = TK::load_a(a.val, vbase + ((int64_t)(ss * MT + t) * 64 + lane) * KPL);
      }
    }
  };

  AFrag acur[KCMAX][MTW], anext[KCMAX][MTW];
  gather(0);
  load_a(0, acur);
  stage_write();
  __syncthreads();
  for (int ch = 0; ch < n_chunks; ++ch) {
    const bool more = ch + 1 < n_chunks;
    if (more) {
      gather(ch + 1);
      load_a(ch + 1, anext);
    }
    const int steps_here = min(KC, n_steps - ch * KC);
#pragma unroll
    for (int sl = 0; sl < KCMAX; ++sl) {
      if (sl < steps_here) {
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
#pragma unroll
          for (int h = 0; h < H; ++h) {
            const BFrag bf = *reinterpret_cast<const BFrag *>(
                stage + ((size_t)((sl * NTB + wn * NT + nt) * H + h) * 64 + lane) * KPL);
#pragma unroll
            for (int m = 0; m < MTW; ++m) acc[m][nt] = TK::mma(acur[sl][m], bf, acc[m][nt]);
          }
        }
      }
    }
    __syncthreads();
    if (more) {
      stage_write();
      __syncthreads();
#pragma unroll
      for (int sl = 0; sl < KCMAX; ++sl)
#pragma unroll
        for (int m = 0; m < MTW; ++m) acur[sl][m] = anext[sl][m];
    }
  }

  // ---- epilogue: v_k (optional) and the K-term fusion into B ----
  const int K = a.K;
  const int lg = lane >> 4, ln = lane & 15;
  const float *gcol = (const float *)a.gcol;
  float *vsave = (float *)a.vsave;
  float *B = (float *)a.B;
  const int wcol = cbase + wn * NT * 16;  // first column of this wave
  if (vsave != nullptr) {
#pragma unroll
    for (int m = 0; m < MTW; ++m)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int c = wcol + nt * 16 + ln;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = (wm * MTW + m) * 16 + 4 * lg + v;
          const int o = b * a.V + row / K, k = row % K;
          if (c < a.C && o < a.N) vsave[((int64_t)k * a.N + o) * a.vs_stride + c] = acc[m][nt][v];
        }
      }
  }
  if (B == nullptr) return;
  if (K == 4 || K == 8 || K == 16) {
    // the K rows of a vertex sit in one or more lane groups of one tile
#pragma unroll
    for (int m = 0; m < MTW; ++m)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int c = wcol + nt * 16 + ln;
        float sum = 0.f;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int k = (4 * lg + v) % K;
          const float gk = (c < a.C) ? gcol[(size_t)k * a.Cs + c] : 0.f;
          sum = fmaf(gk, acc[m][nt][v], sum);
        }
        if (K >= 8) sum += __shfl_xor(sum, 16, 64);
        if (K >= 16) sum += __shfl_xor(sum, 32, 64);
        const bool leader = ((lg * 4) % K) == 0;
        const int o = b * a.V + ((wm * MTW + m) * 16 + 4 * lg) / K;
        if (leader && c < a.C && o < a.N) {
          const int q = c / 3, chn = c - 3 * q;
          B[((int64_t)q * a.N + a.perm[o]) * 3 + chn] = sum;
        }
      }
  } else {
    // generic K: weighted rows through LDS, then sums over the K rows
    float *out = reinterpret_cast<float *>(smem);  // [R][NTB*16]
    const int CW = NTB * 16;
#pragma unroll
    for (int m = 0; m < MTW; ++m)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int cl = wn * NT * 16 + nt * 16 + ln;
        const int c = cbase + cl;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = (wm * MTW + m) * 16 + 4 * lg + v;
          const int k = row % K;
          const float gk = (c < a.C) ? gcol[(size_t)k * a.Cs + c] : 0.f;
          out[row * CW + cl] = gk * acc[m][nt][v];
        }
      }
    __syncthreads();
    for (int idx = threadIdx.x; idx < a.V * CW; idx += nthr) {
      const int vl = idx / CW, cl = idx % CW;
      const int o = b * a.V + vl, c = cbase + cl;
      if (o < a.N && c < a.C) {
        float sum = 0.f;
        for (int k = 0; k < K; ++k) sum += out[(vl * K + k) * CW + cl];
        const int q = c / 3, chn = c - 3 * q;
        B[((int64_t)q * a.N + a.perm[o]) * 3 + chn] = sum;
      }
    }
  }
}

template <int KIND, int MTW, int NT, int KCMAX>
static hipError_t tiles_go(TileArgs a, int nt_total, hipStream_t st) {
  typedef TileKind<KIND> TK;
  const int MT = a.R / 16;
  if (MT % MTW) return hipErrorInvalidValue;
  const int WM = MT / MTW;
  a.wn = 1;
  const int threads = WM * 64;
  const size_t per_step = (size_t)NT * TK::H * 64 * TK::KPL * sizeof(typename TK::BElem);
  int kc = (int)std::min<size_t>(TILE_LDS / per_step, (size_t)TILE_IPT * threads / (64 * NT));
  kc = std::max(1, std::min(kc, KCMAX));
  a.kc = kc;
  const bool reg_epi = a.K == 4 || a.K == 8 || a.K == 16;
  const size_t lds = std::max((size_t)kc * per_step,
                              reg_epi ? (size_t)0 : (size_t)a.R * NT * 16 * sizeof(float));
  const int ngroups = (nt_total + NT - 1) / NT;
  const int hw = ((a.n_blocks + 7) / 8) * 8;
  hipLaunchKernelGGL((k_tiles<KIND, MTW, NT, KCMAX>), dim3(hw, ngroups), dim3(threads), lds, st, a);
  return hipGetLastError();
}

// Shapes: float32 tiles keep one m-tile per wave and stage up to 16 short
// k-steps per chunk; 16-bit tiles give each wave two (or three) m-tiles and
// stage up to 4 k-steps of 32 entries.
template <int KIND>
static hipError_t tiles_kind(const TileArgs &a, hipStream_t st) {
  const int nt = (a.C + 15) / 16;
  const int MT = a.R / 16;
  const int ntw = nt < 3 ? nt : 3;
  if constexpr (KIND == 0) {
    if (ntw == 1) return tiles_go<KIND, 1, 1, 16>(a, nt, st);
    if (ntw == 2) return tiles_go<KIND, 1, 2, 16>(a, nt, st);
    return tiles_go<KIND, 1, 3, 16>(a, nt, st);
  } else {
  if (MT == 6) {
    if (ntw == 1) return tiles_go<KIND, 3, 1, 4>(a, nt, st);
    if (ntw == 2) return tiles_go<KIND, 3, 2, 4>(a, nt, st);
    return tiles_go<KIND, 3, 3, 4>(a, nt, st);
  }
  if (ntw == 1) return tiles_go<KIND, 2, 1, 4>(a, nt, st);
  if (ntw == 2) return tiles_go<KIND, 2, 2, 4>(a, nt, st);
  return tiles_go<KIND, 2, 3, 4>(a, nt, st);
  }
}

int tile_kstep(int vdt) { return vdt == 1 ? 4 : 32; }

hipError_t launch_tiles(const TileArgs &a, int vdt, hipStream_t st) {
  if (a.R % 16 != 0 || a.R < 64 || a.R > 128 || a.n_blocks <= 0) return hipErrorInvalidValue;
  switch (vdt) {
    case 1: return tiles_kind<0>(a, st);
    case 2: return tiles_kind<1>(a, st);
    case 3: return tiles_kind<2>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tlt
