// Wavelet-sparse transport with K-term fusion (Eq. 7 and 8,
// rendering Steps 2 and 4 of Sec. 4), streamed row by row.
//
// The rows (o, k) of the transport are contiguous in memory (row = o*K+k),
// so the whole operator is one stream of (column, value) pairs.  Every wave
// takes an equal contiguous range of rows (+-1 row) and walks it in steps of
// 64*EPL entries: each lane gathers the CPL columns [c0, c0+CPL) of the
// irradiance rows Ehat[j] its entries name and accumulates in registers.
// The gathers of step i are issued before the (non-temporal) loads of step
// i+1, so the HBM latency of the next step overlaps the L2 latency of this
// one without an in-order wait on the prefetch.  At the end of a row the
// lane folds g_k into its running radiance; at the end of a vertex the wave
// reduces once and stores B in original vertex order.  A vertex whose rows
// straddle two waves is cleared by the prep launch and completed with two
// atomic adds, which commute exactly (0 + a + b), so results stay
// deterministic.  The number of waves never exceeds N, so each wave holds
// >= K rows and no vertex spans more than two waves.

#include "device_common.h"

namespace tlt {

template <typename VT, typename CT, int CPL, int EPL, bool NT>
__global__ __launch_bounds__(256) void k_stream(StreamArgs a) {
  const int lb = xcd_remap(blockIdx.x, a.n_logical_blocks);
  if (lb >= a.n_logical_blocks) return;
  const int wave = lb * 4 + (threadIdx.x >> 6);
  if (wave >= a.n_waves) return;
  const int lane = threadIdx.x & 63;
  const int64_t qr = a.R / a.n_waves, rem = a.R % a.n_waves;
  const int64_t r0 = (int64_t)wave * qr + min((int64_t)wave, rem);
  const int64_t r1 = r0 + qr + (wave < rem ? 1 : 0);
  const int c0 = blockIdx.y * CPL;
  const int K = a.K;
  const int n_keep = a.n_keep;
  constexpr int CHUNK = 64 * EPL;
  const int spr = (n_keep + CHUNK - 1) / CHUNK;
  const int32_t *__restrict__ col = a.col;
  const VT *__restrict__ val = (const VT *)a.val;
  const CT *__restrict__ ehat = (const CT *)a.ehat;
  const CT *__restrict__ gcol = (const CT *)a.gcol;
  CT *__restrict__ B = (CT *)a.B;
  CT *__restrict__ vsave = (CT *)a.vsave;
  const bool split_first = (r0 % K) != 0;
  const bool split_last = (r1 % K) != 0;

  // Branch-free prefetch: indices are clamped into the wave's rows and the
  // weights of entries past the row end are zeroed when consumed, so every
  // lane issues the same loads and the wait counts stay exact.
  int jn[EPL];
  CT wn[EPL];
  auto fetch = [&](int64_t r, int s) {
    const int64_t rr = r < r1 ? r : r1 - 1;
#pragma unroll
    for (int u = 0; u < EPL; ++u) {
      const int e = min(s * CHUNK + lane + 64 * u, n_keep - 1);
      const int64_t idx = rr * n_keep + e;
      if constexpr (NT) {
        jn[u] = __builtin_nontemporal_load(col + idx);
        wn[u] = ld_nt<VT, CT>(val, idx);
      } else {
        jn[u] = col[idx];
        wn[u] = ld<VT, CT>(val, idx);
      }
    }
  };

  CT acc[CPL], bacc[CPL];
#pragma unroll
  for (int c = 0; c < CPL; ++c) {
    acc[c] = 0;
    bacc[c] = 0;
  }
  fetch(r0, 0);
  int64_t r = r0;
  int s = 0;
  while (r < r1) {
    int jc[EPL];
    CT wc[EPL];
#pragma unroll
    for (int u = 0; u < EPL; ++u) {
      jc[u] = jn[u];
      wc[u] = (s * CHUNK + lane + 64 * u < n_keep) ? wn[u] : CT(0);
    }
    int64_t rn = r;
    int sn = s + 1;
    if (sn == spr) {
      sn = 0;
      rn = r + 1;
    }
    CT ev[EPL][CPL];
#pragma unroll
    for (int u = 0; u < EPL; ++u) RowLoad<CT, CPL>::load(ehat + (int64_t)jc[u] * a.Cs + c0, ev[u]);
    fetch(rn, sn);
#pragma unroll
    for (int u = 0; u < EPL; ++u)
#pragma unroll
      for (int c = 0; c < CPL; ++c) acc[c] = fma(wc[u], ev[u][c], acc[c]);

    if (sn == 0) {  // row r complete
      const int k = (int)(r % K);
      const int64_t o = r / K;
      const CT *gk = gcol + (size_t)k * a.Cs + c0;
#pragma unroll
      for (int c = 0; c < CPL; ++c) bacc[c] = fma(gk[c], acc[c], bacc[c]);
      if (vsave != nullptr) {
        CT mine = 0;
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
          const CT t = wave_sum(acc[c]);
          if (lane == c) mine = t;
        }
        if (lane < CPL) vsave[((int64_t)a.perm[o] * K + k) * a.vs_stride + c0 + lane] = mine;
      }
#pragma unroll
      for (int c = 0; c < CPL; ++c) acc[c] = 0;
      if (k == K - 1 || r + 1 == r1) {  // vertex complete (or range end)
        if (B != nullptr) {
          CT mine = 0;
#pragma unroll
          for (int c = 0; c < CPL; ++c) {
            const CT t = wave_sum(bacc[c]);
            if (lane == c) mine = t;
          }
          const int c = c0 + lane;
          if (lane < CPL && c < a.C) {
            const int q = c / 3, ch = c - 3 * q;
            const int64_t bi = ((int64_t)q * a.N + a.perm[o]) * 3 + ch;
            const bool split = (split_first && o == r0 / K) || (split_last && r + 1 == r1);
            if (split)
              atomicAdd(&B[bi], mine);
            else
              B[bi] = mine;
          }
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) bacc[c] = 0;
      }
    }
    r = rn;
    s = sn;
  }
}

// ---------------------------------------------------------------------------
// Launch: tile (CPL columns per lane, EPL entries per lane and step) and the
// wave count.
// ---------------------------------------------------------------------------

#define TLT_STREAM_CPL(X) X(4) X(8) X(12) X(16) X(24) X(28) X(32) X(36) X(48) X(64)

bool stream_cpl_supported(int cpl) {
  switch (cpl) {
#define CASE(n) case n: return true;
    TLT_STREAM_CPL(CASE)
#undef CASE
    default: return false;
  }
}

// entries per lane per step: larger for narrow rows to keep enough bytes in
// flight, small for wide rows to bound registers.
constexpr int stream_epl(int cpl) { return cpl <= 4 ? 8 : (cpl <= 8 ? 4 : (cpl <= 16 ? 2 : 1)); }

template <typename VT, typename CT, int CPL, int EPL, bool NT>
static hipError_t stream_go(const StreamArgs &a, int n_chunks, hipStream_t st) {
  const int hw = ((a.n_logical_blocks + 7) / 8) * 8;
  TLT_LAUNCH((k_stream<VT, CT, CPL, EPL, NT>), dim3(hw, n_chunks), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename VT, typename CT>
static hipError_t stream_dispatch(int cpl, const StreamArgs &a, int n_chunks, hipStream_t st) {
  if (cpl == 4) {  // narrow rows: entries per lane and load flavour are tunable
    const int e = a.epl > 0 ? a.epl : 8;
    if (a.nt) {
      if (e == 4) return stream_go<VT, CT, 4, 4, true>(a, n_chunks, st);
      if (e == 16) return stream_go<VT, CT, 4, 16, true>(a, n_chunks, st);
      return stream_go<VT, CT, 4, 8, true>(a, n_chunks, st);
    }
    if (e == 4) return stream_go<VT, CT, 4, 4, false>(a, n_chunks, st);
    if (e == 16) return stream_go<VT, CT, 4, 16, false>(a, n_chunks, st);
    return stream_go<VT, CT, 4, 8, false>(a, n_chunks, st);
  }
  switch (cpl) {
#define CASE(n) \
  case n: return stream_go<VT, CT, n, stream_epl(n), true>(a, n_chunks, st);
    TLT_STREAM_CPL(CASE)
#undef CASE
    default: return hipErrorInvalidValue;
  }
}

int stream_waves(int N, int K, int waves_per_cu) {
  const int64_t cap = (int64_t)256 * (waves_per_cu > 0 ? waves_per_cu : 32);
  int64_t w = std::min<int64_t>(cap, N);
  (void)K;
  return (int)std::max<int64_t>(1, w);
}

hipError_t launch_stream(StreamArgs a, int vdt, bool fp64, int cpl, hipStream_t st) {
  const int n_chunks = (a.C + cpl - 1) / cpl;
  a.n_logical_blocks = (a.n_waves + 3) / 4;
  if (fp64) {
    if (vdt != 0) return hipErrorInvalidValue;
    return stream_dispatch<double, double>(cpl, a, n_chunks, st);
  }
  switch (vdt) {
    case 1: return stream_dispatch<float, float>(cpl, a, n_chunks, st);
    case 2: return stream_dispatch<bf16s, float>(cpl, a, n_chunks, st);
    case 3: return stream_dispatch<f16s, float>(cpl, a, n_chunks, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace tlt
