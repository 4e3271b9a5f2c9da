// Load-time construction of the transport on the device: precompute Step 1
// (listed at the end of Sec. 3.2) -- for every output vertex o and basis term k the kernel row
// btilde_k(|x_o - x_i|) over the Morton-ordered vertices, its orthonormal
// Haar transform (Eq. 8) and the n_keep coefficients of largest magnitude
// (ties to the lower column) -- followed by the block-dense tiles of the
// transport kernel.  Everything is float64 until the final store, and the
// arithmetic is written operation for operation like the host builder
// (no fused multiply-adds), so both produce the same rows.
//
// Selection.  A row of n_cols coefficients never exists in memory: a
// workgroup regenerates the rows of one vertex (all k of its group) in
// chunks of 4096 columns, pass after pass.  Each pass is a step of an exact
// radix select on the compound key (|w| as an ordered integer, then the
// inverted column index), 9 bits at a time: a histogram of the entries
// inside the current key range tells which bin holds the n_keep-th largest
// entry; the range narrows to that bin.  Once the range holds at most CAP
// entries, one more pass writes every entry above the range and keeps the
// range's entries in LDS, where they are ranked exactly.  Histogram and
// counter updates are aggregated per wave (one atomic per distinct bin),
// because neighbouring coefficients of one level fall in the same bins.
// The kept entries are written unordered, then sorted by column per row.

#include "device_common.h"

namespace tlt {

namespace {

constexpr int BT = 512;         // threads per workgroup
constexpr int CPT = 8;          // columns per thread and chunk
constexpr int CH = BT * CPT;    // columns per chunk
constexpr int NBIN = 512;       // 9-bit digits
constexpr int CAP = 96;         // candidates ranked in LDS per row
constexpr int NDIG = 11;        // 7 digits of |w| (63 bits) + 4 of the column (31 bits)
constexpr int KG_MAX = 8;

// A row histograms (HIST) until its key range holds at most CAP entries,
// collects (COLLECT) in the next pass, has its candidates ranked at the end
// of that pass (RANK), and is then DONE.  Untruncated rows take ALL entries
// in a single pass.
enum { PH_HIST = 0, PH_COLLECT = 1, PH_DONE = 2, PH_ALL = 3, PH_RANK = 4 };

struct KState {
  uint64_t lo_w, hi_w;    // current key range (|w| bits)
  uint32_t lo_j, hi_j;    // current range of 0x7fffffff - column
  int phase, digit;
  int above;              // entries known to rank above the range
  int need;               // entries still to take from the range
};

__device__ __forceinline__ int digit_shift(int d) {
  return d < 7 ? 54 - 9 * d : (d == 7 ? 22 : d == 8 ? 13 : d == 9 ? 4 : 0);
}
__device__ __forceinline__ int digit_bins(int d) { return d == 10 ? 16 : NBIN; }
__device__ __forceinline__ int digit_of(int d, uint64_t kw, uint32_t kj) {
  const int sh = digit_shift(d);
  return d < 7 ? (int)((kw >> sh) & 511u) : (int)((kj >> sh) & (uint32_t)(digit_bins(d) - 1));
}

__device__ __forceinline__ uint64_t lanes_below() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// base[key] += 1 for every active lane, one atomic per distinct key.
__device__ __forceinline__ void agg_count(uint32_t *base, int key, bool act) {
  uint64_t m = __ballot(act);
  const int lane = threadIdx.x & 63;
  while (m) {
    const int leader = __ffsll((unsigned long long)m) - 1;
    const int k0 = __shfl(key, leader, 64);
    const uint64_t same = __ballot(act && key == k0);
    if (lane == leader) atomicAdd(&base[k0], (uint32_t)__popcll(same));
    m &= ~same;
  }
}

// Like agg_count, and returns each active lane's own slot (old value plus
// its rank among the lanes of the same key).
__device__ __forceinline__ int agg_slot(uint32_t *base, int key, bool act) {
  uint64_t m = __ballot(act);
  const int lane = threadIdx.x & 63;
  const uint64_t lt = lanes_below();
  int slot = 0;
  while (m) {
    const int leader = __ffsll((unsigned long long)m) - 1;
    const int k0 = __shfl(key, leader, 64);
    const uint64_t same = __ballot(act && key == k0);
    uint32_t old = 0;
    if (lane == leader) old = atomicAdd(&base[k0], (uint32_t)__popcll(same));
    old = __shfl(old, leader, 64);
    if (act && key == k0) slot = (int)old + __popcll(same & lt);
    m &= ~same;
  }
  return slot;
}

__device__ __forceinline__ void store_value(void *val, int vdt, int64_t i, double v) {
  switch (vdt) {
    case 0: ((double *)val)[i] = v; break;
    case 1: ((float *)val)[i] = (float)v; break;
    case 2: ((uint16_t *)val)[i] = to_bf16((float)v); break;
    default: ((uint16_t *)val)[i] = __builtin_bit_cast(uint16_t, (_Float16)(float)v); break;
  }
}

// BF16 rounding of what the BF16 storage of v leaves out (v - bf16(v)).
__device__ __forceinline__ uint16_t bf16_residual(double v) {
  const float hi = __uint_as_float((uint32_t)to_bf16((float)v) << 16);
  return to_bf16((float)(v - (double)hi));
}

// Caller-given float64 rows (load time): entries e0 .. e0+n of the rows
// rounded to storage, and for BF16 tiles the residual words of the columns
// below head_cols, exactly as the device build stores them.
__global__ void k_quantize_rows(const double *__restrict__ src, const int32_t *__restrict__ col,
                                void *__restrict__ val, int vdt, int64_t e0, int64_t n,
                                int64_t n_keep, uint16_t *__restrict__ res, int head_cols) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t e = e0 + i;
  const double w = src[i];
  store_value(val, vdt, e, w);
  if (res != nullptr) {
    const int j = col[e];
    if (j < head_cols) res[e / n_keep * head_cols + j] = bf16_residual(w);
  }
}

struct Shared {
  double *rn;          // [nr]
  double2 *bs;         // [KG][nr] (basis, slope)
  double *lv;          // [KG][BT] level values inside a chunk
  double *cs;          // [KG][max_chunks] chunk scaling coefficients
  uint32_t *hc;        // [KG][NBIN] histogram, or the candidates of a collecting row
  uint32_t *outc;      // [KG] entries written in the collect pass
  uint32_t *candc;     // [KG] candidates kept in the collect pass
  KState *st;          // [KG]
};

// Candidate storage inside a row's histogram region (NBIN words).
__device__ __forceinline__ uint64_t *cand_w(uint32_t *hc, int k) {
  return reinterpret_cast<uint64_t *>(hc + (size_t)k * NBIN);
}
__device__ __forceinline__ double *cand_v(uint32_t *hc, int k) {
  return reinterpret_cast<double *>(hc + (size_t)k * NBIN) + CAP;
}
__device__ __forceinline__ int32_t *cand_j(uint32_t *hc, int k) {
  return reinterpret_cast<int32_t *>(hc + (size_t)k * NBIN + 4 * CAP);
}

// One generated coefficient w at column j of row (vertex, k).  Must be
// called by every lane of the wave (inactive lanes pass valid = false);
// k may differ between lanes.
__device__ __forceinline__ void entry(const BuildArgs &a, const Shared &sh, const KState &s, int v,
                                      int k, int j, double w, bool valid, int *bad) {
  const int ph = valid ? s.phase : PH_DONE;
  const uint64_t kw = (uint64_t)__double_as_longlong(w) & 0x7fffffffffffffffull;
  const uint32_t kj = 0x7fffffffu - (uint32_t)j;
  const bool in = kw >= s.lo_w && kw <= s.hi_w && kj >= s.lo_j && kj <= s.hi_j;
  const bool up = kw > s.hi_w || (kw >= s.lo_w && kj > s.hi_j);
  // histogram pass
  const bool h = ph == PH_HIST && in;
  agg_count(sh.hc, k * NBIN + (h ? digit_of(s.digit, kw, kj) : 0), h);
  // collect pass: entries above the range are kept, the range's are ranked
  const bool tk = ph == PH_COLLECT && up;
  const int slot = agg_slot(sh.outc, k, tk);
  if (tk) {
    if (slot < s.above) {
      const int64_t r = ((int64_t)v * a.K + a.kg0 + k) * a.n_keep + slot;
      a.scol[r] = j;
      a.sval[r] = w;
    } else {
      *bad = 1;
    }
  }
  const bool cd = ph == PH_COLLECT && in;
  const int cs = agg_slot(sh.candc, k, cd);
  if (cd) {
    if (cs < CAP) {
      cand_w(sh.hc, k)[cs] = kw;
      cand_v(sh.hc, k)[cs] = w;
      cand_j(sh.hc, k)[cs] = j;
    } else {
      *bad = 1;
    }
  }
  // untruncated rows: every coefficient at its own column
  if (ph == PH_ALL) {
    const int64_t r = ((int64_t)(a.o0 + v) * a.K + a.kg0 + k) * a.n_keep + j;
    a.col[r] = j;
    store_value(a.val, a.vdt, r, w);
    if (a.res != nullptr && j < a.head_cols)
      a.res[((int64_t)(a.o0 + v) * a.K + a.kg0 + k) * a.head_cols + j] = bf16_residual(w);
  }
}

// Haar levels l0+1, l0+2, ... over the n values buf[k*stride + 0..n) of
// every row of the group (in place, sums to the front) until one value is
// left, reporting each detail: detail p of level l of block `blk` sits at
// column (n_cols >> l) + blk * (details per block at l) + p.
__device__ __forceinline__ void lds_levels(const BuildArgs &a, const Shared &sh, int v, int KG,
                                           double *buf, int stride, int n, int l0, int64_t blk,
                                           double hsq, int *bad) {
  const int t = threadIdx.x;
  for (int l = l0 + 1; n > 1; ++l) {
    const int half = n >> 1;
    const int total = KG * half;
    constexpr int MAXIT = KG_MAX * (CH / 16) / BT;  // items per thread at the widest level
    double sv[MAXIT], dv[MAXIT];
    int kk[MAXIT], pp[MAXIT];
    bool ok[MAXIT];
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
      const int item = it * BT + t;
      ok[it] = item < total;
      kk[it] = ok[it] ? item / half : 0;
      pp[it] = ok[it] ? item % half : 0;
      if (ok[it]) {
        const double x0 = buf[kk[it] * stride + 2 * pp[it]];
        const double x1 = buf[kk[it] * stride + 2 * pp[it] + 1];
        dv[it] = (x0 - x1) * hsq;
        sv[it] = (x0 + x1) * hsq;
      } else {
        dv[it] = 0.0;
        sv[it] = 0.0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int it = 0; it < MAXIT; ++it) {
      if (it * BT < total) {  // uniform
        if (ok[it]) buf[kk[it] * stride + pp[it]] = sv[it];
        const int j = (int)((a.n_cols >> l) + blk * half + pp[it]);
        const KState s = sh.st[kk[it]];
        entry(a, sh, s, v, kk[it], j, dv[it], ok[it], bad);
      }
    }
    __syncthreads();
    n = half;
  }
}

}  // namespace

// grid: nv vertices (one workgroup each).  KG = number of k of this launch.
template <int KG>
__global__ __launch_bounds__(BT) void k_build_select(BuildArgs a) {
#pragma clang fp contract(off)
  extern __shared__ __align__(16) unsigned char smem[];
  Shared sh;
  {
    unsigned char *p = smem;
    sh.st = reinterpret_cast<KState *>(p);
    p += sizeof(KState) * KG_MAX;
    sh.outc = reinterpret_cast<uint32_t *>(p);
    p += sizeof(uint32_t) * KG_MAX;
    sh.candc = reinterpret_cast<uint32_t *>(p);
    p += sizeof(uint32_t) * KG_MAX;
    p = smem + ((p - smem + 15) / 16) * 16;
    sh.hc = reinterpret_cast<uint32_t *>(p);
    p += sizeof(uint32_t) * NBIN * KG;
    sh.lv = reinterpret_cast<double *>(p);
    p += sizeof(double) * BT * KG;
    sh.cs = reinterpret_cast<double *>(p);
    p += sizeof(double) * ((a.max_chunks * KG + 1) / 2 * 2);  // keeps bs 16-byte aligned
    sh.bs = reinterpret_cast<double2 *>(p);
    p += sizeof(double2) * a.nr * KG;
    sh.rn = reinterpret_cast<double *>(p);
  }
  const int t = threadIdx.x;
  const int v = blockIdx.x;        // vertex of this launch's range
  const int o = a.o0 + v;          // Morton position of the output vertex
  const int nr = a.nr;
  const int N = a.N;
  const bool haar = a.haar != 0;
  const double hsq = a.hsq;
  int bad = 0;

  for (int i = t; i < nr; i += BT) sh.rn[i] = a.rn[i];
  for (int i = t; i < nr * KG; i += BT) {
    const int k = a.kg0 + i / nr, m = i % nr;
    sh.bs[i] = double2{a.basis[(size_t)k * nr + m], a.slope[(size_t)k * nr + m]};
  }
  if (t < KG) {
    KState s;
    s.lo_w = 0;
    s.hi_w = 0x7fffffffffffffffull;
    s.lo_j = 0;
    s.hi_j = 0x7fffffffu;
    s.phase = a.all ? PH_ALL : PH_HIST;
    s.digit = 0;
    s.above = 0;
    s.need = 0;
    sh.st[t] = s;
  }
  const double xo = a.pos[3 * (size_t)o], yo = a.pos[3 * (size_t)o + 1], zo = a.pos[3 * (size_t)o + 2];
  const int chw = a.n_cols < CH ? a.n_cols : CH;            // columns per chunk
  const int n_chunks = (a.n_cols + chw - 1) / chw;
  int lc = 0;                                                // Haar levels inside a chunk
  while ((1 << lc) < chw) ++lc;
  __syncthreads();

  for (int pass = 0; pass <= NDIG + 1; ++pass) {
    // prepare the pass; stop when every row is done
    bool any = false;
    for (int k = 0; k < KG; ++k) any |= sh.st[k].phase != PH_DONE;
    if (!any) break;
    for (int i = t; i < KG * NBIN; i += BT) {
      if (sh.st[i / NBIN].phase == PH_HIST) sh.hc[i] = 0u;
    }
    if (t < KG) {
      sh.outc[t] = 0u;
      sh.candc[t] = 0u;
    }
    __syncthreads();

    for (int c = 0; c < n_chunks; ++c) {
      const int c0 = c * chw;
      // this thread's CPT columns: distance, node and offset
      int node[CPT];
      double dr[CPT];
      bool live[CPT];   // a column of the row (plain form) / a vertex (Haar)
#pragma unroll
      for (int q = 0; q < CPT; ++q) {
        const int i = c0 + t * CPT + q;
        live[q] = (t * CPT + q < chw) && i < N;
        node[q] = 0;
        dr[q] = 0.0;
        if (live[q]) {
          const double dx = xo - a.pos[3 * (size_t)i];
          const double dy = yo - a.pos[3 * (size_t)i + 1];
          const double dz = zo - a.pos[3 * (size_t)i + 2];
          const double r = sqrt(dx * dx + dy * dy + dz * dz);
          int m;
          if (r >= sh.rn[nr - 1]) {
            m = nr - 1;
          } else if (r <= 0.0) {
            m = 0;
          } else {
            m = (int)((nr - 1) * sqrt(r / sh.rn[nr - 1]));
            if (m > nr - 2) m = nr - 2;
            if (m < 0) m = 0;
            while (m > 0 && r < sh.rn[m]) --m;
            while (m < nr - 2 && r >= sh.rn[m + 1]) ++m;
          }
          node[q] = m;
          dr[q] = r - sh.rn[m];
        }
      }
      const bool tin = t * CPT < chw;   // thread holds columns of this chunk
      for (int k = 0; k < KG; ++k) {
        const KState s = sh.st[k];
        if (s.phase == PH_DONE) continue;  // uniform
        double x[CPT];
#pragma unroll
        for (int q = 0; q < CPT; ++q) {
          x[q] = 0.0;
          if (live[q]) {
            const int m = node[q];
            const double2 b = sh.bs[k * nr + m];
            x[q] = (m == nr - 1) ? sh.bs[k * nr + nr - 1].x : b.y * dr[q] + b.x;
          }
        }
        if (haar) {
          // levels 1..3 in registers (chw >= 8)
          double s1[4], s2[2];
#pragma unroll
          for (int p = 0; p < 4; ++p) {
            const double d = (x[2 * p] - x[2 * p + 1]) * hsq;
            s1[p] = (x[2 * p] + x[2 * p + 1]) * hsq;
            entry(a, sh, s, v, k, (a.n_cols >> 1) + (c0 >> 1) + 4 * t + p, d, tin, &bad);
          }
#pragma unroll
          for (int p = 0; p < 2; ++p) {
            const double d = (s1[2 * p] - s1[2 * p + 1]) * hsq;
            s2[p] = (s1[2 * p] + s1[2 * p + 1]) * hsq;
            entry(a, sh, s, v, k, (a.n_cols >> 2) + (c0 >> 2) + 2 * t + p, d, tin, &bad);
          }
          {
            const double d = (s2[0] - s2[1]) * hsq;
            const double s3 = (s2[0] + s2[1]) * hsq;
            entry(a, sh, s, v, k, (a.n_cols >> 3) + (c0 >> 3) + t, d, tin, &bad);
            if (tin) sh.lv[k * BT + t] = s3;
          }
        } else {
#pragma unroll
          for (int q = 0; q < CPT; ++q) {
            const int i = c0 + t * CPT + q;
            entry(a, sh, s, v, k, i, x[q], (t * CPT + q < chw) && i < a.n_cols, &bad);
          }
        }
      }
      if (haar) {
        __syncthreads();
        // levels 4..lc over the chunk's chw/8 level-3 sums
        lds_levels(a, sh, v, KG, sh.lv, BT, chw >> 3, 3, c, hsq, &bad);
        if (t < KG) sh.cs[t * a.max_chunks + c] = sh.lv[t * BT];
      }
      __syncthreads();
    }
    if (haar) {
      // coarse levels over the chunk sums, then the scaling coefficient
      if (n_chunks > 1) lds_levels(a, sh, v, KG, sh.cs, a.max_chunks, n_chunks, lc, 0, hsq, &bad);
      const int k0 = t < KG ? t : 0;
      const KState s0 = sh.st[k0];
      entry(a, sh, s0, v, k0, 0, sh.cs[k0 * a.max_chunks], t < KG, &bad);
      __syncthreads();
    }

    // close the pass
    if (t < KG) {
      KState s = sh.st[t];
      if (s.phase == PH_HIST) {
        const int nb = digit_bins(s.digit);
        int acc = s.above, b = nb - 1;
        for (; b > 0; --b) {
          const int hb = (int)sh.hc[t * NBIN + b];
          if (acc + hb >= a.n_keep) break;
          acc += hb;
        }
        const int cnt = (int)sh.hc[t * NBIN + b];
        if (acc + cnt < a.n_keep) bad = 1;  // fewer entries than n_keep in range
        const int shf = digit_shift(s.digit);
        if (s.digit < 7) {
          s.lo_w = (s.lo_w & ~(511ull << shf)) | ((uint64_t)b << shf);
          s.hi_w = s.lo_w | ((1ull << shf) - 1ull);
        } else {
          const uint32_t mk = (uint32_t)(nb - 1);
          s.lo_j = (s.lo_j & ~(mk << shf)) | ((uint32_t)b << shf);
          s.hi_j = s.lo_j | ((1u << shf) - 1u);
        }
        s.above = acc;
        s.need = a.n_keep - acc;
        if (cnt <= CAP) {
          s.phase = PH_COLLECT;
        } else if (s.digit + 1 >= NDIG) {
          bad = 1;
          s.phase = PH_DONE;
        } else {
          s.digit += 1;
        }
        sh.st[t] = s;
      } else if (s.phase == PH_ALL) {
        s.phase = PH_DONE;
        sh.st[t] = s;
      } else if (s.phase == PH_COLLECT) {
        if ((int)sh.outc[t] != s.above || (int)sh.candc[t] < s.need) bad = 1;
        s.phase = PH_RANK;
        sh.st[t] = s;
      }
    }
    __syncthreads();
    // rank the candidates of the rows that collected in this pass and take
    // the best `need`
    for (int item = t; item < KG * CAP; item += BT) {
      const int k = item / CAP, i = item % CAP;
      const KState s = sh.st[k];
      if (s.phase != PH_RANK) continue;
      const int nc = min((int)sh.candc[k], CAP);
      if (i >= nc) continue;
      const uint64_t wi = cand_w(sh.hc, k)[i];
      const int ji = cand_j(sh.hc, k)[i];
      int rank = 0;
      for (int u = 0; u < nc; ++u) {
        const uint64_t wu = cand_w(sh.hc, k)[u];
        rank += (wu > wi || (wu == wi && cand_j(sh.hc, k)[u] < ji)) ? 1 : 0;
      }
      if (rank < s.need) {
        const int64_t r = ((int64_t)v * a.K + a.kg0 + k) * a.n_keep + s.above + rank;
        a.scol[r] = ji;
        a.sval[r] = cand_v(sh.hc, k)[i];
      }
    }
    __syncthreads();
    if (t < KG && sh.st[t].phase == PH_RANK) sh.st[t].phase = PH_DONE;
    __syncthreads();
  }
  if (t < KG && sh.st[t].phase != PH_DONE) bad = 1;
  if (bad) atomicOr(a.status, 1);
}

// Sort the kept entries of each row by column; store columns and values.
template <int P>
__global__ __launch_bounds__(256) void k_build_sort(BuildArgs a) {
  __shared__ uint64_t key[P];
  const int r = blockIdx.x;                       // row of this launch's range
  const int64_t g = (int64_t)a.o0 * a.K + r;      // global row
  const int n = (int)a.n_keep;
  const int t = threadIdx.x;
  for (int i = t; i < P; i += 256)
    key[i] = i < n ? (((uint64_t)(uint32_t)a.scol[(int64_t)r * n + i] << 32) | (uint32_t)i) : ~0ull;
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      __syncthreads();
      for (int i = t; i < P / 2; i += 256) {
        const int lo = 2 * stride * (i / stride) + (i % stride);
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t x = key[lo], y = key[hi];
        if ((x > y) == asc) {
          key[lo] = y;
          key[hi] = x;
        }
      }
    }
  }
  __syncthreads();
  for (int i = t; i < n; i += 256) {
    const uint64_t kk = key[i];
    const int slot = (int)(kk & 0xffffffffu);
    const int j = (int)(kk >> 32);
    const double w = a.sval[(int64_t)r * n + slot];
    a.col[g * n + i] = j;
    store_value(a.val, a.vdt, g * n + i, w);
    if (a.res != nullptr && j < a.head_cols) a.res[g * a.head_cols + j] = bf16_residual(w);
    if (i > 0 && (key[i - 1] >> 32) >= (kk >> 32)) atomicOr(a.status, 2);
  }
}

// ---------------------------------------------------------------------------
// Fragment-sparse tiles from the (column, value) rows.  Per block (one
// workgroup): the union of the kept columns of its rows as a bitmap; the
// union entries (and, with residuals, the head columns once more); the
// m-tiles (16-row groups, rows ordered (k, o)) that keep each entry; the
// entries ordered by (first m-tile, last m-tile, entry) so that the entries
// kept by the same m-tiles sit in the same k-steps; then, per k-step, the
// mask of m-tiles with a kept entry in it.  Only those (k-step, m-tile)
// fragments are stored.  The count pass gives the padded entry count and
// the fragment count of every block, the fill pass (same ordering) writes
// the union ids, the masks and the values.  Unions above TB_UL entries
// (or with ordering off) keep column order and store every fragment.
// ---------------------------------------------------------------------------

constexpr int TB_UL = 8192;   // largest union ordered by m-tile pattern

constexpr int TB_STEPS = TB_UL / 4;   // k-steps of an ordered union (k-step >= 4)

// LDS layout of the build: bm, pref [n_words] u32; then, when ordering,
// pat [TB_UL/2] u32 (16-bit patterns), key [TB_UL] u32, pos [TB_UL/2] u32
// (16-bit positions), mask [TB_STEPS] u16, fpref [TB_STEPS] u32 (fragments
// before each step).
size_t tile_build_lds(int n_words, bool order) {
  size_t b = 2 * sizeof(uint32_t) * (size_t)n_words;
  if (order) b += sizeof(uint32_t) * (TB_UL / 2 + TB_UL + TB_UL / 2) + 6 * TB_STEPS;
  return b;
}

struct TileOrder {
  uint32_t *bm, *pref, *pat, *key, *pos, *fpref;
  uint16_t *mask;
  int U0, H, U, n_steps, MT;
  bool ordered;
  uint32_t frags;   // fragments stored
};

// Column of union entry e (< U0 + H) from the bitmap: the e-th set bit
// (entries >= U0 are the residuals of the first entries).  Only used for
// the few head entries.
__device__ __forceinline__ int union_col_of(const TileOrder &o, const TileBuildArgs &a, int e) {
  if (e >= o.U0) e -= o.U0;
  for (int w = 0; w < a.n_words; ++w) {
    const int c = __popc(o.bm[w]);
    if (e < c) {
      uint32_t bits = o.bm[w];
      for (int i = 0; i < e; ++i) bits &= bits - 1u;
      return 32 * w + __ffs(bits) - 1;
    }
    e -= c;
  }
  return 0;
}

__device__ __forceinline__ int rank_of(const TileOrder &o, int j) {
  return (int)(o.pref[j >> 5] + (uint32_t)__popc(o.bm[j >> 5] & ((1u << (j & 31)) - 1u)));
}

// Row of the block for vertex offset vl and term k: (k, o) order for
// fragment-sparse tiles, (o, k) for dense ones.
__device__ __forceinline__ int tile_row(const TileBuildArgs &a, int vl, int k) {
  return a.order ? k * a.V + vl : vl * a.K + k;
}

__device__ void block_order(const TileBuildArgs &a, int b, unsigned char *smem, TileOrder &o) {
  const int t = threadIdx.x;
  const int R = a.V * a.K, ks = a.kstep;
  o.MT = R / 16;
  o.bm = reinterpret_cast<uint32_t *>(smem);
  o.pref = o.bm + a.n_words;
  uint32_t *tail = o.pref + a.n_words;
  o.pat = tail;
  o.key = o.pat + TB_UL / 2;
  o.pos = o.key + TB_UL;
  o.mask = reinterpret_cast<uint16_t *>(o.pos + TB_UL / 2);
  o.fpref = reinterpret_cast<uint32_t *>(o.mask + TB_STEPS);
  __shared__ uint32_t tsum[256];
  __shared__ uint32_t s_total, s_frags;
  // bitmap of the kept columns
  for (int w = t; w < a.n_words; w += 256) o.bm[w] = 0u;
  __syncthreads();
  const int v0 = b * a.V, v1 = min(a.N, v0 + a.V);
  const int64_t e0 = (int64_t)v0 * a.K * a.n_keep, e1 = (int64_t)v1 * a.K * a.n_keep;
  for (int64_t e = e0 + t; e < e1; e += 256) {
    const int j = a.col[e];
    atomicOr(&o.bm[j >> 5], 1u << (j & 31));
  }
  __syncthreads();
  // exclusive prefix of the word popcounts: contiguous word ranges per thread
  const int per = (a.n_words + 255) / 256;
  const int w0 = min(a.n_words, t * per), w1 = min(a.n_words, w0 + per);
  uint32_t sum = 0;
  for (int w = w0; w < w1; ++w) sum += (uint32_t)__popc(o.bm[w]);
  tsum[t] = sum;
  __syncthreads();
  if (t == 0) {
    uint32_t acc = 0;
    for (int i = 0; i < 256; ++i) {
      const uint32_t x = tsum[i];
      tsum[i] = acc;
      acc += x;
    }
    s_total = acc;
  }
  __syncthreads();
  sum = tsum[t];
  for (int w = w0; w < w1; ++w) {
    o.pref[w] = sum;
    sum += (uint32_t)__popc(o.bm[w]);
  }
  o.U0 = (int)s_total;
  // residual entries: the union's columns below head_cols (its first H entries)
  o.H = 0;
  if (a.res != nullptr)
    for (int w = 0; w * 32 < a.head_cols; ++w) {
      const int nb = min(32, a.head_cols - 32 * w);
      o.H += __popc(o.bm[w] & (nb == 32 ? 0xffffffffu : ((1u << nb) - 1u)));
    }
  o.U = o.U0 + o.H;
  o.n_steps = (o.U + ks - 1) / ks;
  o.ordered = a.order && o.U <= TB_UL && o.MT <= 16;
  __syncthreads();
  if (!o.ordered) {
    o.frags = (uint32_t)o.n_steps * o.MT;
    return;
  }
  // m-tile patterns of the entries (16 bits each, two per word)
  for (int i = t; i < TB_UL / 2; i += 256) o.pat[i] = 0u;
  __syncthreads();
  for (int64_t e = e0 + t; e < e1; e += 256) {
    const int j = a.col[e];
    const int rk = (int)((e - e0) / a.n_keep);            // (o, k) row of the input
    const int r = tile_row(a, rk / a.K, rk % a.K);
    const int u = rank_of(o, j);
    atomicOr(&o.pat[u >> 1], (1u << (r >> 4)) << (16 * (u & 1)));
  }
  __syncthreads();
  auto pat_of = [&](int e) -> uint32_t {
    const int u = e >= o.U0 ? e - o.U0 : e;
    return (o.pat[u >> 1] >> (16 * (u & 1))) & 0xffffu;
  };
  // sort keys (first m-tile, last m-tile, entry), padded to a power of two
  int P2 = 1;
  while (P2 < o.U) P2 <<= 1;
  for (int i = t; i < P2; i += 256) {
    uint32_t k = 0xffffffffu;
    if (i < o.U) {
      const uint32_t pt = pat_of(i);
      const uint32_t first = (uint32_t)__ffs(pt) - 1u, last = 31u - (uint32_t)__clz(pt);
      k = ((first * 16u + last) << 20) | (uint32_t)i;
    }
    o.key[i] = k;
  }
  __syncthreads();
  for (int kk = 2; kk <= P2; kk <<= 1) {
    for (int jj = kk >> 1; jj > 0; jj >>= 1) {
      for (int i = t; i < P2; i += 256) {
        const int l = i ^ jj;
        if (l > i) {
          const uint32_t x = o.key[i], y = o.key[l];
          const bool asc = (i & kk) == 0;
          if ((x > y) == asc) {
            o.key[i] = y;
            o.key[l] = x;
          }
        }
      }
      __syncthreads();
    }
  }
  // position of every entry; mask of every k-step
  for (int i = t; i < TB_UL / 2; i += 256) o.pos[i] = 0u;
  __syncthreads();
  for (int p = t; p < o.U; p += 256) {
    const int e = (int)(o.key[p] & 0xfffffu);
    atomicOr(&o.pos[e >> 1], (uint32_t)p << (16 * (e & 1)));
  }
  for (int s = t; s < o.n_steps; s += 256) {
    uint32_t m = 0;
    for (int p = s * ks; p < min(o.U, (s + 1) * ks); ++p) m |= pat_of((int)(o.key[p] & 0xfffffu));
    o.mask[s] = (uint16_t)m;
  }
  __syncthreads();
  if (t == 0) {
    uint32_t acc = 0;
    for (int s = 0; s < o.n_steps; ++s) {
      o.fpref[s] = acc;
      acc += (uint32_t)__popc((uint32_t)o.mask[s]);
    }
    s_frags = acc;
  }
  __syncthreads();
  o.frags = s_frags;
}

__device__ __forceinline__ int pos_of(const TileOrder &o, int e) {
  return o.ordered ? (int)((o.pos[e >> 1] >> (16 * (e & 1))) & 0xffffu) : e;
}

__global__ __launch_bounds__(256) void k_tile_count(TileBuildArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  TileOrder o;
  block_order(a, blockIdx.x, smem, o);
  if (threadIdx.x == 0) {
    a.count[blockIdx.x] = (int64_t)o.n_steps * a.kstep;
    a.fcount[blockIdx.x] = (int64_t)o.frags;
  }
}

__global__ __launch_bounds__(256) void k_tile_fill(TileBuildArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  TileOrder o;
  const int b = blockIdx.x;
  const int t = threadIdx.x;
  block_order(a, b, smem, o);
  const int64_t off = a.blk_off[b];
  const int64_t nu = a.blk_off[b + 1] - off;           // n_steps * kstep
  const int64_t fo = a.frag_off[b];
  const uint32_t nf = (uint32_t)(a.frag_off[b + 1] - fo);
  const int ks = a.kstep, kpl = ks / 4, MT = o.MT;
  // union ids at their positions; padding entries read column 0
  const int per = (a.n_words + 255) / 256;
  const int w0 = min(a.n_words, t * per), w1 = min(a.n_words, w0 + per);
  for (int w = w0; w < w1; ++w) {
    uint32_t bits = o.bm[w];
    int u = (int)o.pref[w];
    while (bits) {
      const int bit = __ffs(bits) - 1;
      const int p = pos_of(o, u);
      if (p < nu) a.ucol[off + p] = 32 * w + bit;
      ++u;
      bits &= bits - 1u;
    }
  }
  for (int h = t; h < o.H; h += 256) {
    const int p = pos_of(o, o.U0 + h);
    if (p < nu) a.ucol[off + p] = union_col_of(o, a, h);
  }
  for (int64_t p = o.U + t; p < nu; p += 256) a.ucol[off + p] = 0;
  // step masks
  const int64_t s0 = off / ks;
  for (int s = t; s < o.n_steps; s += 256)
    a.mask[s0 + s] = o.ordered ? o.mask[s] : (uint16_t)((1u << MT) - 1u);
  // values: fragment (step, m-tile) stored at its rank among the block's
  // stored fragments; lane l holds rows 16 m + l % 16, elements
  // kpl (l / 16) .. of the step
  const int v0 = b * a.V, v1 = min(a.N, v0 + a.V);
  const int64_t e0 = (int64_t)v0 * a.K * a.n_keep, e1 = (int64_t)v1 * a.K * a.n_keep;
  auto put = [&](int p, int r, uint32_t word) {
    const int st = p / ks, rem = p % ks, m = r >> 4;
    uint32_t f;
    if (o.ordered) {
      const uint32_t msk = o.mask[st];
      if (!((msk >> m) & 1u)) return;   // cannot happen: the entry's pattern has bit m
      f = o.fpref[st] + (uint32_t)__popc(msk & ((1u << m) - 1u));
    } else {
      f = (uint32_t)st * MT + m;
    }
    if (f >= nf) return;
    const int lane = (rem / kpl) * 16 + (r & 15);
    const int64_t w = ((fo + f) * 64 + lane) * kpl + rem % kpl;
    if (a.esz == 4)
      ((uint32_t *)a.tval)[w] = word;
    else
      ((uint16_t *)a.tval)[w] = (uint16_t)word;
  };
  for (int64_t e = e0 + t; e < e1; e += 256) {
    const int j = a.col[e];
    const int rk = (int)((e - e0) / a.n_keep);
    const int r = tile_row(a, rk / a.K, rk % a.K);
    const int u = rank_of(o, j);
    const uint32_t word = a.esz == 4 ? ((const uint32_t *)a.val)[e] : ((const uint16_t *)a.val)[e];
    put(pos_of(o, u), r, word);
    if (a.res != nullptr && j < a.head_cols)   // u < H: the residual entry U0 + u
      put(pos_of(o, o.U0 + u), r, a.res[e / a.n_keep * a.head_cols + j]);
  }
}

// ---------------------------------------------------------------------------
// Launches.
// ---------------------------------------------------------------------------

size_t build_select_lds(int KG, int nr, int max_chunks) {
  size_t p = sizeof(KState) * KG_MAX + 2 * sizeof(uint32_t) * KG_MAX;
  p = (p + 15) / 16 * 16;
  p += sizeof(uint32_t) * NBIN * KG + sizeof(double) * BT * KG +
       sizeof(double) * ((max_chunks * KG + 1) / 2 * 2) + sizeof(double2) * nr * KG + sizeof(double) * nr;
  return p;
}

int build_chunk_columns() { return CH; }
int build_max_group() { return KG_MAX; }

hipError_t launch_build_select(const BuildArgs &a, int KG, hipStream_t st) {
  if (KG < 1 || KG > KG_MAX || a.nv < 1) return hipErrorInvalidValue;
  const size_t lds = build_select_lds(KG, a.nr, a.max_chunks);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  switch (KG) {
#define CASE(n) \
  case n: hipLaunchKernelGGL(k_build_select<n>, dim3(a.nv), dim3(BT), lds, st, a); break;
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(7) CASE(8)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_build_sort(const BuildArgs &a, hipStream_t st) {
  const int64_t rows = (int64_t)a.nv * a.K;
  int P = 64;
  while (P < a.n_keep) P <<= 1;
  switch (P) {
#define CASE(n) \
  case n: hipLaunchKernelGGL(k_build_sort<n>, dim3((unsigned)rows), dim3(256), 0, st, a); break;
    CASE(64) CASE(128) CASE(256) CASE(512) CASE(1024) CASE(2048) CASE(4096) CASE(8192)
#undef CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int build_sort_max() { return 8192; }

hipError_t launch_quantize_rows(const double *src, const int32_t *col, void *val, int vdt, int64_t e0,
                                int64_t n, int64_t n_keep, uint16_t *res, int head_cols, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_quantize_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, col, val,
                     vdt, e0, n, n_keep, res, head_cols);
  return hipGetLastError();
}

hipError_t launch_tile_count(const TileBuildArgs &a, hipStream_t st) {
  const size_t lds = tile_build_lds(a.n_words, a.order);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tile_count, dim3(a.n_blocks), dim3(256), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_tile_fill(const TileBuildArgs &a, hipStream_t st) {
  const size_t lds = tile_build_lds(a.n_words, a.order);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_tile_fill, dim3(a.n_blocks), dim3(256), lds, st, a);
  return hipGetLastError();
}

}  // namespace tlt
