// Block-dense tiles: the wavelet-sparse transport of Eq. (7)/(8)
// (rendering Steps 2 and 4 of Sec. 4) as 16x16 matrix-instruction tiles.
//
// A block holds the R = V*K rows of V Morton-consecutive vertices, ordered
// (k, o), over the union U of their kept columns, ordered so that entries
// kept by the same rows share k-steps.  Only the (k-step, 16-row m-tile)
// fragments holding a kept coefficient are stored (dense inside: about
// half of their slots are kept coefficients, the rest zeros); a 16-bit mask
// per k-step says which.  One workgroup per block (and 16*NT-column group),
// waves split the m-tiles:
//
//   D[row, c] = sum_u W[row, u] * Ehat[U[u], c]       (MFMA, FP32 accumulate)
//   B[o, c]   = sum_k g_k[c] * D[(k,o), c]            (K-term fusion)
//
// W streams from HBM once, in fragment order (one contiguous 256 B or 1 KB
// load per wave, step and stored m-tile; absent fragments are loads past
// the block's buffer range, which return zeros without a memory access,
// and their matrix instructions are skipped).  The gathered irradiance rows Ehat[U[u]] are
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

#include <type_traits>

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
  static constexpr int VSZ = 4;  // bytes per stored value
  template <int AUX>
  static __device__ __forceinline__ AFrag frag(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX));
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
  static constexpr int VSZ = 2;
  template <int AUX>
  static __device__ __forceinline__ AFrag frag(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(AFrag, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
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
  static constexpr int VSZ = 2;
  template <int AUX>
  static __device__ __forceinline__ AFrag frag(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(AFrag, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, AUX));
  }
  static __device__ __forceinline__ void split(float x, BElem &hi, BElem &lo) {
    hi = (_Float16)x;
    lo = (_Float16)(x - (float)hi);
  }
};

// Work split: a workgroup owns one block and one group of NT <= 3 16-column
// tiles (wider launches run as several column groups).  Its WM = MT/MTW
// waves each compute MTW m-tiles x NT n-tiles.  The gathered irradiance of
// up to `chunk` union entries is staged in LDS (B-operand fragment order) in
// one pass and read by every wave -- for narrow launches the whole union of
// a block fits one chunk, so the block synchronises once.  W streams through
// a PD-deep register ring per wave (fragments PD steps ahead of use), which
// runs across chunk boundaries, so HBM latency hides behind PD steps of
// matrix work regardless of the staging.
constexpr int TILE_LDS = 64 * 1024;  // staging budget per workgroup

// CGS: float32 tiles stage each (step, lane group) row of B with this
// compile-time stride (>= the group's real columns), so the per-step LDS
// offsets are immediates.
// CSC: k-steps per staged chunk, a compile-time multiple of PD, so the
// matrix work of a chunk is straight-line code and the load counters can
// be waited on exactly.
// WAUX: cache policy of the W loads -- 2 (non-temporal) when the tile
// values exceed the Infinity Cache and a block is read by one column group
// only (W then streams past the caches, which keep the gathered irradiance
// rows: measured 2062 -> 1936 us at 163842 vertices, 48 columns), else 0:
// several column groups re-read a block through L2 (non-temporal measured
// 624 -> 694 us at 40962 vertices, 192 columns in three groups), and tiles
// that fit the Infinity Cache stay there from one render to the next
// (non-temporal measured 41.8 -> 44.7 us at 10242 vertices, 232 MB).
// SP: fragment-sparse blocks (rows (k, o), entries in m-tile pattern order,
// only fragments with a kept coefficient stored, per-step masks); else
// dense blocks (rows (o, k), entries in column order, every fragment
// stored, the K rows of a vertex fused in registers).
template <int KIND, int MTW, int NT, int PD, int IPT, int CGS, int CSC, int WAUX, bool SP>
__global__ __launch_bounds__(512) void k_tiles(TileArgs a) {
  typedef TileKind<KIND> TK;
  typedef typename TK::BElem BElem;
  typedef typename TK::BFrag BFrag;
  typedef typename TK::AFrag AFrag;
  constexpr int KS = TK::KSTEP, KPL = TK::KPL, H = TK::H;
  extern __shared__ __align__(16) unsigned char smem[];
  BElem *stage = reinterpret_cast<BElem *>(smem);

  // Workgroup h runs on XCD h % 8.  Each XCD takes a contiguous range of
  // blocks, and the column groups of one block occupy consecutive slots of
  // the same XCD, so they run together and share the W block through L2.
  const int ng = a.n_groups;
  const int per_xcd = idx::tile_per_xcd(a.n_blocks);
  const int b = idx::tile_block(blockIdx.x, per_xcd, ng);
  const int grp = idx::tile_group(blockIdx.x, ng);
  if (!idx::tile_runs(blockIdx.x, per_xcd, ng, a.n_blocks)) return;
  const int lane = threadIdx.x & 63;
  // waves split the m-tiles; the sparse form branches on the wave's m-tiles,
  // so its wave index is made a scalar
  const int wave = SP ? __builtin_amdgcn_readfirstlane(threadIdx.x >> 6) : (int)(threadIdx.x >> 6);
  const int wm = wave;
  const int nthr = blockDim.x;
  const int cbase = grp * NT * 16;
  const int cg = min(NT * 16, a.C - cbase);  // real columns of this group
  const int64_t u0 = a.blk_off[b];
  const int n_steps = (int)((a.blk_off[b + 1] - u0) / KS);
  const int64_t f0 = a.foff[b];
  const int n_frags = (int)(a.foff[b + 1] - f0);
  constexpr int CS = CSC;
  const int32_t *__restrict__ ucol = a.ucol + u0;
  const float *__restrict__ ehat = (const float *)a.ehat;

  // Staging.  The union column ids of the whole block are read into LDS
  // once.  float32: item = (step sl, lane group lg, real column n), one
  // 4-byte gather and store.  16-bit kinds: item = (step, lane group, column
  // quad), eight 16-byte gathers of (hi|lo) words -- 4 columns of KPL = 8
  // consecutive union entries -- unpacked into 2 x 4 fragment stores.  A
  // thread's item decomposition is the same for every chunk.  The gathers
  // of the next chunk are issued into registers before the current chunk's
  // matrix work and stored to LDS after it.
  int *uc = reinterpret_cast<int *>(smem + a.uc_offset);
  uint16_t *mk = reinterpret_cast<uint16_t *>(smem + a.mk_offset);
  for (int i = threadIdx.x; i < n_steps * KS; i += nthr) uc[i] = ucol[i];
  if constexpr (SP)
    for (int i = threadIdx.x; i < n_steps; i += nthr) mk[i] = a.fmask[u0 / KS + i];
  constexpr int QW = KIND == 0 ? 1 : 4;  // columns per item
  const int cq = (cg + QW - 1) / QW;     // items per (step, lane group)
  int it_sl[IPT], it_eoff[IPT], it_col[IPT], it_lds[IPT], it_slot[IPT], it_sw[IPT];
#pragma unroll
  for (int it = 0; it < IPT; ++it) {
    const int item = threadIdx.x + it * nthr;
    const int q = item % cq;
    const int lg = (item / cq) % 4;
    const int sl = item / (cq * 4);
    const int n = q * QW;
    it_sl[it] = sl;
    it_eoff[it] = sl * KS + KPL * lg;
    it_col[it] = cbase + n;
    if constexpr (KIND == 0)
      it_lds[it] = (sl * 4 + lg) * CGS + n;
    else
    {
      // fragment base, lane slot of the first of the item's four columns,
      // and the slot swizzle of this (column tile, lane group): see read_b
      it_lds[it] = (sl * NT + n / 16) * H * 64 * KPL;
      it_slot[it] = idx::tile_stage_lane(n, lg);
      it_sw[it] = idx::tile_stage_swizzle(n, lg);
    }
  }
  __syncthreads();  // union ids visible
  typedef typename std::conditional<KIND == 0, float, uint4>::type GT;
  const GT *__restrict__ esrc = (const GT *)(KIND == 0 ? a.ehat : a.ehat2);
  GT g[IPT][KPL];
  auto gather = [&](int s0, int ns) {
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      const bool ok = it_sl[it] < ns;
#pragma unroll
      for (int i = 0; i < KPL; ++i) {
        const int j = ok ? uc[s0 * KS + it_eoff[it] + i] : 0;
        const int64_t idx = (int64_t)j * a.Cs + (ok ? it_col[it] : 0);
        if constexpr (KIND == 0)
          g[it][i] = esrc[idx];
        else
          g[it][i] = *(const uint4 *)((const uint32_t *)esrc + idx);
      }
    }
  };
  auto stage_write = [&](int ns) {
#pragma unroll
    for (int it = 0; it < IPT; ++it) {
      if (it_sl[it] < ns) {
        if constexpr (KIND == 0) {
          stage[it_lds[it]] = g[it][0];
        } else {
#pragma unroll
          for (int jj = 0; jj < 4; ++jj) {
            uint32_t hw[KPL / 2], lw[KPL / 2];
#pragma unroll
            for (int i = 0; i < KPL / 2; ++i) {
              const uint32_t w0 = g[it][2 * i][jj], w1 = g[it][2 * i + 1][jj];
              hw[i] = __builtin_amdgcn_perm(w1, w0, 0x05040100u);
              lw[i] = __builtin_amdgcn_perm(w1, w0, 0x07060302u);
            }
            const int ph = idx::tile_stage_slot(it_slot[it], jj, it_sw[it]) * KPL;
            *reinterpret_cast<BFrag *>(stage + it_lds[it] + ph) = __builtin_bit_cast(BFrag, hw);
            *reinterpret_cast<BFrag *>(stage + it_lds[it] + ph + 64 * KPL) =
                __builtin_bit_cast(BFrag, lw);
          }
        }
      }
    }
  };
  // 16-bit kinds: padded columns of the group read zeros, clear the buffer
  if (KIND != 0 && cg < NT * 16) {
    const int words = CS * NT * H * 64 * KPL * (int)sizeof(BElem) / 4;
    for (int i = threadIdx.x; i < words; i += nthr) reinterpret_cast<uint32_t *>(smem)[i] = 0u;
    __syncthreads();
  }

  f32x4 acc[MTW][NT];
#pragma unroll
  for (int m = 0; m < MTW; ++m)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) acc[m][nt] = f32x4{0, 0, 0, 0};

  // W fragments of this wave's m-tiles, step by step, through a buffer
  // resource over the block's stored fragments.  The loads run in step order
  // at a frontier PD steps ahead of the matrix work; fp_load counts the
  // stored fragments of the steps before the frontier, so the fragment of
  // (step s, m-tile t) is number fp_load + popcount(mask[s] below t).  An
  // absent fragment (and every step past the block's end, whose mask reads
  // as 0) gets an offset past the range, which the buffer bound turns into
  // zeros without a memory access.  All offsets are in the vector operand,
  // which the range check covers.  The masks of the 64 steps from the
  // current chunk's first one sit one per lane in a register (cm) and are
  // taken out with a scalar lane read: the frontier of chunk step sl is
  // step sl + PD < 64 of the window (16-bit chunks hold at most 16 steps).
  constexpr int FRAG = 64 * KPL * TK::VSZ;   // bytes per stored fragment
  constexpr int OOB = 0x7ffff000;
  const __amdgpu_buffer_rsrc_t wrs = __builtin_amdgcn_make_buffer_rsrc(
      (void *)((const char *)a.val + f0 * FRAG), (short)0, n_frags * FRAG, 0x00020000);
  const int lane_off = lane * KPL * TK::VSZ;
  const int tbase = wm * MTW;   // this wave's first m-tile
  uint32_t fp_load = 0;
  int s_load = 0;
  const int MT = a.R / 16;
  uint32_t cm = 0;
  auto mask_window = [&](int s0) {
    if constexpr (SP) cm = s0 + lane < n_steps ? (uint32_t)mk[s0 + lane] : 0u;
  };
  auto win = [&](int i) -> uint32_t { return (uint32_t)__builtin_amdgcn_readlane((int)cm, i); };
  // ms: the mask of the frontier step (sparse form only)
  auto load_next = [&](AFrag (&dst)[MTW], uint32_t ms) {
    if constexpr (SP) {
#pragma unroll
      for (int m = 0; m < MTW; ++m) {
        const int t = tbase + m;
        const uint32_t idx = fp_load + (uint32_t)__popc(ms & ((1u << t) - 1u));
        const int voff = ((ms >> t) & 1u) ? (int)(idx * FRAG) + lane_off : OOB;
        dst[m] = TK::template frag<WAUX>(wrs, voff, 0);
      }
      fp_load += (uint32_t)__popc(ms);
    } else {
      // every fragment stored: (s, t) is number s MT + t.  The step is a
      // scalar offset, the lane a fixed vector offset.  Steps past the
      // block's end (the ring runs up to CS + PD - 1 of them ahead) reload
      // its last step: they only ever multiply zero B fragments, and every
      // read stays inside the block.
      const int sc = min(s_load, n_steps - 1);
#pragma unroll
      for (int m = 0; m < MTW; ++m)
        dst[m] = TK::template frag<WAUX>(wrs, (tbase + m) * FRAG + lane_off, sc * MT * FRAG);
    }
    ++s_load;
  };
  // B fragments of step sl of the staged chunk (unconditional LDS reads).
  // 16-bit kinds: the fragment of (step, column tile nt, half h) holds lane
  // l's 16 bytes at slot idx::tile_read_slot(l, nt), a permutation inside
  // groups of four slots that keeps both these reads and the staging
  // stores (each thread writes one column quad, four consecutive slots, for
  // consecutive (column quad, lane group) items) free of bank conflicts.
  auto read_b = [&](int sl, BFrag (&dst)[NT][H]) {
#pragma unroll
    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
      for (int h = 0; h < H; ++h) {
        if constexpr (KIND == 0) {
          const int n = nt * 16 + (lane & 15);
          const float v = stage[((size_t)sl * 4 + (lane >> 4)) * CGS + min(n, cg - 1)];
          dst[nt][h] = n < cg ? v : 0.f;
        } else {
          const int slot = idx::tile_read_slot(lane, nt);
          dst[nt][h] = *reinterpret_cast<const BFrag *>(
              stage + ((size_t)((sl * NT + nt) * H + h) * 64 + slot) * KPL);
        }
      }
  };
  AFrag ring[PD][MTW];
  if constexpr (SP) {
    static_assert(!SP || KIND != 0, "fragment-sparse tiles are 16-bit");
    __syncthreads();  // step masks visible
  }
  mask_window(0);
#pragma unroll
  for (int p = 0; p < PD; ++p) load_next(ring[p], SP ? win(p) : 0u);

  int ns = min(CS, n_steps);
  gather(0, ns);
  stage_write(ns);
  __syncthreads();
  for (int s0 = 0; s0 < n_steps; s0 += CS) {
    const int nxt = s0 + CS;
    const int ns_next = min(CS, n_steps - nxt);
    if (ns_next > 0) gather(nxt, ns_next);
    if (s0 > 0) mask_window(s0);
    // sparse blocks: the B operands of a step are read one step ahead, into
    // two buffers taken in turn by step parity (compile-time indices; at
    // large-f16-163842 1474 -> 1455 us).  Dense blocks read them at their
    // step: the extra registers cost their 128-row launches occupancy
    // (batch64-bf16-40962: 570 -> 672 us).
    BFrag bfs[2][NT][H];
    if constexpr (SP) {
      if (((win(0) >> tbase) & ((1u << MTW) - 1u)) != 0u) read_b(0, bfs[0]);
    }
    // Groups of PD steps: a group runs whole or not at all, so the W ring
    // stays in step (one refill per step, in step order) and the load
    // counters can be waited on exactly.  16-bit kinds run every group of a
    // chunk, also past the block's end in its last chunk (those steps
    // multiply zero B fragments, or have an empty mask), so the number of
    // loads issued per chunk is a compile-time constant: the staging of the
    // next chunk then waits for its gathered rows only, not for the W ring
    // (with a runtime group count the compiler waited for every load, and
    // the ring drained at each chunk: batch64-bf16-40962 562 -> 546 us in
    // one sweep).
    // Float32 chunks hold up to 256 steps and keep the runtime bound.  A
    // step whose mask has none of the wave's m-tiles (absent fragments, and
    // steps past the block's end, whose mask is 0) skips its operand reads
    // and matrix work; only its refill runs.
#pragma unroll
    for (int g0 = 0; g0 < CS; g0 += PD) {
      if (KIND != 0 || g0 < ns) {
        float bg[KIND == 0 ? PD : 1];
        if constexpr (KIND == 0) {
          const int n = lane & 15;
          const float *sp = stage + (size_t)g0 * 4 * CGS + (lane >> 4) * CGS + min(n, cg - 1);
#pragma unroll
          for (int p = 0; p < PD; ++p) bg[p] = sp[p * 4 * CGS];
#pragma unroll
          for (int p = 0; p < PD; ++p) bg[p] = (n < cg && g0 + p < ns) ? bg[p] : 0.f;
        }
#pragma unroll
        for (int p = 0; p < PD; ++p) {
          const int sl = g0 + p;
          if constexpr (SP) {
            // scalar: this wave's m-tiles stored at this step and the next
            const uint32_t wb = (win(sl) >> tbase) & ((1u << MTW) - 1u);
            const uint32_t wbn = sl + 1 < CS ? (win(sl + 1) >> tbase) & ((1u << MTW) - 1u) : 0u;
            if (wbn != 0u) read_b(sl + 1, bfs[(sl + 1) & 1]);   // then sl + 1 < ns
            if (wb != 0u) {   // then sl < ns
              BFrag (&bf)[NT][H] = bfs[sl & 1];
              if (wb == (1u << MTW) - 1u) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                  for (int h = 0; h < H; ++h)
#pragma unroll
                    for (int m = 0; m < MTW; ++m) acc[m][nt] = TK::mma(ring[p][m], bf[nt][h], acc[m][nt]);
              } else {
#pragma unroll
                for (int m = 0; m < MTW; ++m)
                  if ((wb >> m) & 1u) {
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                      for (int h = 0; h < H; ++h) acc[m][nt] = TK::mma(ring[p][m], bf[nt][h], acc[m][nt]);
                  }
              }
            }
          } else {
            // dense: steps of the last group past the chunk's end multiply
            // zero B fragments
            BFrag bf[NT][H];
            if constexpr (KIND == 0) {
              bf[0][0] = bg[p];
            } else {
              read_b(min(sl, ns - 1), bf);
              if (sl >= ns) {
#pragma unroll
                for (int nt = 0; nt < NT; ++nt)
#pragma unroll
                  for (int h = 0; h < H; ++h) bf[nt][h] = BFrag{};
              }
            }
#pragma unroll
            for (int nt = 0; nt < NT; ++nt)
#pragma unroll
              for (int h = 0; h < H; ++h)
#pragma unroll
                for (int m = 0; m < MTW; ++m) acc[m][nt] = TK::mma(ring[p][m], bf[nt][h], acc[m][nt]);
          }
          load_next(ring[p], SP ? win(sl + PD) : 0u);  // refill this slot PD steps ahead
          // keep the refill right behind its step (no regrouping of loads)
          __builtin_amdgcn_sched_barrier(0);
        }
      }
    }
    if (ns_next > 0) {
      __syncthreads();  // every wave is done with this chunk
      stage_write(ns_next);
      __syncthreads();
    }
    ns = ns_next;
  }

  // ---- epilogue.  Sparse blocks: rows r = k V + vl; dense blocks: rows
  // r = vl K + k.  v_k (optional; row (perm[o], k) of vsave, vertices in
  // original order), then the K-term fusion: B[o, c] = sum over k in order
  // of g_k[c] D[(o, k), c] -- in registers when the K rows of a vertex sit
  // in lane groups of one m-tile (dense blocks, K = 4, 8, 16), else through
  // LDS.
  const int K = a.K, V = a.V;
  const int lg = lane >> 4, ln = lane & 15;
  const float *gcol = (const float *)a.gcol;
  float *vsave = (float *)a.vsave;
  float *B = (float *)a.B;
  constexpr int CW = NT * 16;
  auto row_k = [&](int r) { return SP ? r / V : r % K; };
  auto row_v = [&](int r) { return SP ? r % V : r / K; };
  if (vsave != nullptr) {
#pragma unroll
    for (int m = 0; m < MTW; ++m)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int c = cbase + nt * 16 + ln;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int r = (tbase + m) * 16 + 4 * lg + v;
          const int o = b * V + row_v(r);
          if (c < a.C && o < a.N)
            vsave[((int64_t)a.perm[o] * K + row_k(r)) * a.vs_stride + c] = acc[m][nt][v];
        }
      }
  }
  if (B == nullptr) return;
  if (!SP && (K == 4 || K == 8 || K == 16)) {
#pragma unroll
    for (int m = 0; m < MTW; ++m)
#pragma unroll
      for (int nt = 0; nt < NT; ++nt) {
        const int c = cbase + nt * 16 + ln;
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
        const int o = b * V + ((tbase + m) * 16 + 4 * lg) / K;
        if (leader && c < a.C && o < a.N) {
          const int q = c / 3, chn = c - 3 * q;
          B[((int64_t)q * a.N + a.perm[o]) * 3 + chn] = sum;
        }
      }
    return;
  }
  __syncthreads();   // every wave is done with the staged chunk
  float *out = reinterpret_cast<float *>(smem);  // [R][CW]
#pragma unroll
  for (int m = 0; m < MTW; ++m)
#pragma unroll
    for (int nt = 0; nt < NT; ++nt) {
      const int cl = nt * 16 + ln;
      const int c = cbase + cl;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = (tbase + m) * 16 + 4 * lg + v;
        out[r * CW + cl] = (c < a.C ? gcol[(size_t)row_k(r) * a.Cs + c] : 0.f) * acc[m][nt][v];
      }
    }
  __syncthreads();
  for (int idx = threadIdx.x; idx < V * CW; idx += nthr) {
    const int vl = idx / CW, cl = idx % CW;
    const int o = b * V + vl, c = cbase + cl;
    if (o < a.N && c < a.C) {
      float sum = 0.f;
      for (int k = 0; k < K; ++k) sum += out[(SP ? k * V + vl : vl * K + k) * CW + cl];
      const int q = c / 3, chn = c - 3 * q;
      B[((int64_t)q * a.N + a.perm[o]) * 3 + chn] = sum;
    }
  }
}

template <int KIND, int MTW, int NT, int PD, int IPT, int CGS, int CSC>
static hipError_t tiles_launch(TileArgs a, size_t per_step, hipStream_t st) {
  const int threads = (a.R / 16 / MTW) * 64;
  a.kc = CSC;
  a.wn = 1;
  // the staging buffer also holds the epilogue's weighted rows [R][NT*16]
  // when they are summed through LDS
  const bool reg_epi = !a.sparse && (a.K == 4 || a.K == 8 || a.K == 16);
  size_t stage = std::max((size_t)CSC * per_step, reg_epi ? (size_t)0 : (size_t)a.R * NT * 16 * sizeof(float));
  stage = (stage + 15) / 16 * 16;
  a.uc_offset = (int)stage;
  const size_t masks = stage + sizeof(int) * (size_t)a.max_union;
  a.mk_offset = (int)masks;
  const size_t lds =
      masks + (a.sparse ? (sizeof(uint16_t) * (size_t)(a.max_union / TileKind<KIND>::KSTEP) + 15) / 16 * 16 : 0);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  // (dense blocks clamp the ring's step to the block's last one, so every
  // W read stays inside the block)
  const int hw = 8 * ((a.n_blocks + 7) / 8) * a.n_groups;
  const bool nt_w = a.n_groups == 1 && a.stream_w;
  if constexpr (KIND == 0) {
    if (a.sparse) return hipErrorInvalidValue;   // fragment-sparse tiles are 16-bit
  } else {
    // the mask window covers the ring's reach: CSC - 1 + PD < 64
    static_assert(CSC + PD <= 64, "mask window");
    if (a.sparse && nt_w) {
      TLT_LAUNCH((k_tiles<KIND, MTW, NT, PD, IPT, CGS, CSC, 2, true>), dim3(hw), dim3(threads), lds, st, a);
      return hipGetLastError();
    }
    if (a.sparse) {
      TLT_LAUNCH((k_tiles<KIND, MTW, NT, PD, IPT, CGS, CSC, 0, true>), dim3(hw), dim3(threads), lds, st, a);
      return hipGetLastError();
    }
  }
  if (nt_w)
    TLT_LAUNCH((k_tiles<KIND, MTW, NT, PD, IPT, CGS, CSC, 2, false>), dim3(hw), dim3(threads), lds, st, a);
  else
    TLT_LAUNCH((k_tiles<KIND, MTW, NT, PD, IPT, CGS, CSC, 0, false>), dim3(hw), dim3(threads), lds, st, a);
  return hipGetLastError();
}

template <int KIND, int MTW, int NT, int PD, int IPT, int CGS = 16>
static hipError_t tiles_go(TileArgs a, int nt_total, hipStream_t st) {
  typedef TileKind<KIND> TK;
  const int MT = a.R / 16;
  if (MT % MTW) return hipErrorInvalidValue;
  const int threads = (MT / MTW) * 64;
  const int cmax = std::min(a.C, NT * 16);  // real columns of the widest group
  const int qw = KIND == 0 ? 1 : 4;
  const int items_per_step = 4 * ((cmax + qw - 1) / qw);
  if (KIND == 0 && cmax > CGS) return hipErrorInvalidValue;
  const size_t per_step = KIND == 0 ? (size_t)4 * CGS * sizeof(float)
                                    : (size_t)NT * TK::H * 64 * TK::KPL * sizeof(typename TK::BElem);
  // staging budget: TILE_LDS, or for blocks of 16 m-tiles -- one
  // workgroup of eight waves per CU at their register count -- what the
  // CU's LDS leaves beside the union ids and step masks
  size_t budget = TILE_LDS;
  if (MT == 16) {
    const size_t fixed = sizeof(int) * (size_t)a.max_union +
                         sizeof(uint16_t) * (size_t)(a.max_union / TK::KSTEP) + 64;
    budget = fixed < (size_t)160 * 1024 ? (size_t)160 * 1024 - fixed : 0;
  }
  int cs = std::min<int>((int)(budget / per_step), IPT * threads / items_per_step);
  if (a.kc > 0) cs = std::min(cs, a.kc);  // caller override (tuning)
  if (cs < PD || (size_t)PD * items_per_step > (size_t)IPT * threads) return hipErrorInvalidValue;
  a.n_groups = (nt_total + NT - 1) / NT;
  // the largest compiled chunk length that fits
  if constexpr (KIND == 0) {
    if (cs >= 256) return tiles_launch<KIND, MTW, NT, PD, IPT, CGS, 256>(a, per_step, st);
    if (cs >= 128) return tiles_launch<KIND, MTW, NT, PD, IPT, CGS, 128>(a, per_step, st);
    if (cs >= 64) return tiles_launch<KIND, MTW, NT, PD, IPT, CGS, 64>(a, per_step, st);
    if (cs >= 32) return tiles_launch<KIND, MTW, NT, PD, IPT, CGS, 32>(a, per_step, st);
    return tiles_launch<KIND, MTW, NT, PD, IPT, CGS, 16>(a, per_step, st);
  } else {
    if (cs >= 16) return tiles_launch<KIND, MTW, NT, PD, IPT, CGS, 16>(a, per_step, st);
    if (cs >= 8) return tiles_launch<KIND, MTW, NT, PD, IPT, CGS, 8>(a, per_step, st);
    return tiles_launch<KIND, MTW, NT, PD, IPT, CGS, 4>(a, per_step, st);
  }
}

// Shapes: float32 tiles keep one m-tile per wave, one 16-column tile per
// group, a 16-step W ring and 8 staged items per thread (a narrow union fits
// one chunk); 16-bit tiles use up to three 16-column tiles per group, a
// 4-step ring, one gathered item (4 columns x 8 entries) per thread and
// chunk, and two m-tiles per wave when a block has eight.
template <int KIND>
static hipError_t tiles_kind(const TileArgs &a, hipStream_t st) {
  const int nt = (a.C + 15) / 16;
  const int MT = a.R / 16;
  const int ntw = nt < 3 ? nt : 3;
  if constexpr (KIND == 0) {
    const int cmax = a.C < 16 ? a.C : 16;
    if (cmax <= 4) return tiles_go<KIND, 1, 1, 16, 8, 4>(a, nt, st);
    if (cmax <= 8) return tiles_go<KIND, 1, 1, 16, 8, 8>(a, nt, st);
    return tiles_go<KIND, 1, 1, 16, 8, 16>(a, nt, st);
  } else {
    if (MT == 16) {
      // 256-row blocks (16-bit storage): eight waves of two m-tiles share
      // each staged irradiance row, so the gathered bytes per W byte halve
      // against 128-row blocks
      // With three or four column tiles, chunks of 16 steps (the default,
      // or a chunk cap of 16) take two gathered items per thread.
      if (ntw == 1) return tiles_go<KIND, 2, 1, 4, 1>(a, nt, st);
      if (ntw == 2) return tiles_go<KIND, 2, 2, 4, 1>(a, nt, st);
      const bool two = a.kc == 0 || a.kc >= 16;
      if (a.shape == 241) return two ? tiles_go<KIND, 2, 4, 4, 2>(a, nt, st) : tiles_go<KIND, 2, 4, 4, 1>(a, nt, st);
      return two ? tiles_go<KIND, 2, 3, 4, 2>(a, nt, st) : tiles_go<KIND, 2, 3, 4, 1>(a, nt, st);
    }
    if (MT == 8) {
      // tuned shapes: more m-tiles per wave halve the LDS reads of the
      // staged irradiance per matrix instruction; four n-tiles per group
      // cut the re-reads of W across column groups
      switch (a.shape) {
        case 241: return tiles_go<KIND, 2, 4, 4, 1>(a, nt, st);
        case 432: return tiles_go<KIND, 4, 3, 4, 2>(a, nt, st);
        case 442: return tiles_go<KIND, 4, 4, 4, 2>(a, nt, st);
        default: break;
      }
      if (ntw == 1) return tiles_go<KIND, 2, 1, 4, 1>(a, nt, st);
      if (ntw == 2) return tiles_go<KIND, 2, 2, 4, 1>(a, nt, st);
      return tiles_go<KIND, 2, 3, 4, 1>(a, nt, st);
    }
    if (ntw == 1) return tiles_go<KIND, 1, 1, 4, 1>(a, nt, st);
    if (ntw == 2) return tiles_go<KIND, 1, 2, 4, 1>(a, nt, st);
    return tiles_go<KIND, 1, 3, 4, 1>(a, nt, st);
  }
}

int tile_kstep(int vdt) { return vdt == 1 ? 4 : 32; }

int tile_max_rows(int vdt) { return vdt == 1 ? 128 : 256; }

hipError_t launch_tiles(const TileArgs &a, int vdt, hipStream_t st) {
  if (a.R % 16 != 0 || a.R < 48 || a.R > tile_max_rows(vdt) || a.n_blocks <= 0)
    return hipErrorInvalidValue;
  if (a.R > 128 && a.R != 256) return hipErrorInvalidValue;
  switch (vdt) {
    case 1: return tiles_kind<0>(a, st);
    case 2: return tiles_kind<1>(a, st);
    case 3: return tiles_kind<2>(a, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tlt
