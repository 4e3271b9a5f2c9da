// Host construction of the block-dense transport tiles (load time).
//
// For every block of V Morton-consecutive vertices the kept columns of its
// V*K rows are merged into one sorted union; the rows are then stored
// densely over that union (zeros where a row did not keep the column), in
// the operand order of the 16x16 matrix instructions.  Consecutive vertices
// share most kept columns (the coarse Haar levels and the fine levels near
// them), so about half of the dense slots are kept coefficients and the
// dense block costs no more memory than (index, value) pairs.

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <thread>
#include <vector>

#include "host_internal.h"

namespace tlt {

uint16_t f32_to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

uint16_t f32_to_f16(float f) {
  uint32_t x;
  std::memcpy(&x, &f, 4);
  const uint16_t sign = (uint16_t)((x >> 16) & 0x8000u);
  const uint32_t mant = x & 0x7fffffu;
  const int exp = (int)((x >> 23) & 0xffu);
  if (exp == 0xff) return (uint16_t)(sign | 0x7c00u | (mant ? 0x200u : 0u));
  const int e = exp - 127 + 15;
  if (e >= 31) return (uint16_t)(sign | 0x7c00u);
  if (e >= 1) {
    uint32_t m = mant >> 13;
    const uint32_t rem = mant & 0x1fffu;
    if (rem > 0x1000u || (rem == 0x1000u && (m & 1u))) ++m;
    uint32_t out = ((uint32_t)e << 10) + m;  // a mantissa carry bumps the exponent
    if (out >= 0x7c00u) return (uint16_t)(sign | 0x7c00u);
    return (uint16_t)(sign | out);
  }
  // subnormal result: value = full * 2^(exp - 150), units of 2^-24
  if (exp == 0) return sign;  // float32 subnormals are far below half of 2^-24
  const uint32_t full = mant | 0x800000u;
  const int shift = 126 - exp;  // >= 14
  if (shift > 25) return sign;
  uint32_t m = full >> shift;
  const uint32_t rem = full & ((1u << shift) - 1u);
  const uint32_t half = 1u << (shift - 1);
  if (rem > half || (rem == half && (m & 1u))) ++m;
  return (uint16_t)(sign | m);
}

void tiles_append(TileBuild &tb, int nv, int n_cols, int64_t n_keep, const int32_t *col,
                  const double *val, int vdt, int n_threads) {
  const int V = tb.V, K = tb.K, R = V * K, ks = tb.kstep, kpl = ks / 4;
  const int nb = (nv + V - 1) / V;
  if (tb.blk_off.empty()) tb.blk_off.push_back(0);
  // 1. unions, per block, in parallel
  std::vector<std::vector<int32_t>> U(nb);
  {
    std::atomic<int> next(0);
    auto work = [&]() {
      std::vector<int32_t> tmp;
      for (;;) {
        const int b = next.fetch_add(1);
        if (b >= nb) break;
        const int v0 = b * V, v1 = std::min(nv, v0 + V);
        tmp.assign(col + (size_t)v0 * K * n_keep, col + (size_t)v1 * K * n_keep);
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        const size_t up = (tmp.size() + ks - 1) / ks * ks;
        tmp.resize(up, 0);
        U[b] = tmp;
      }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < n_threads; ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
  }
  const int64_t base_blk = tb.n_blocks;
  std::vector<int64_t> off(nb + 1);
  off[0] = tb.blk_off.back();
  for (int b = 0; b < nb; ++b) off[b + 1] = off[b] + (int64_t)U[b].size();
  tb.blk_off.resize(base_blk + nb + 1);
  for (int b = 0; b <= nb; ++b) tb.blk_off[base_blk + b] = off[b];
  tb.ucol.resize(off[nb]);
  const size_t vbase = (size_t)off[0] * R, vend = (size_t)off[nb] * R;
  if (vdt == TLT_F32)
    tb.v32.resize(vend);
  else
    tb.v16.resize(vend);
  // 2. dense fragment-ordered values, per block, in parallel
  {
    std::atomic<int> next(0);
    auto work = [&]() {
      std::vector<int32_t> loc(n_cols, -1);
      std::vector<double> dense;
      for (;;) {
        const int b = next.fetch_add(1);
        if (b >= nb) break;
        const std::vector<int32_t> &u = U[b];
        const int nu = (int)u.size();
        std::memcpy(&tb.ucol[off[b]], u.data(), sizeof(int32_t) * nu);
        // local index of each real union column (padding entries repeat 0;
        // the first occurrence of a column is the real one)
        for (int i = nu - 1; i >= 0; --i) loc[u[i]] = i;
        dense.assign((size_t)nu * R, 0.0);
        const int v0 = b * V, v1 = std::min(nv, v0 + V);
        for (int v = v0; v < v1; ++v)
          for (int k = 0; k < K; ++k) {
            const int row = (v - v0) * K + k;
            const size_t rb = ((size_t)v * K + k) * n_keep;
            for (int64_t e = 0; e < n_keep; ++e)
              dense[(size_t)loc[col[rb + e]] * R + row] = val[rb + e];
          }
        for (int i = 0; i < nu; ++i) loc[u[i]] = -1;
        // fragment order
        const int steps = nu / ks, mt = R / 16;
        size_t w = (size_t)off[b] * R;
        for (int s = 0; s < steps; ++s)
          for (int t = 0; t < mt; ++t)
            for (int l = 0; l < 64; ++l)
              for (int i = 0; i < kpl; ++i, ++w) {
                const int uu = s * ks + kpl * (l / 16) + i;
                const int row = 16 * t + (l % 16);
                const double x = dense[(size_t)uu * R + row];
                if (vdt == TLT_F32)
                  tb.v32[w] = (float)x;
                else if (vdt == TLT_BF16)
                  tb.v16[w] = f32_to_bf16((float)x);
                else
                  tb.v16[w] = f32_to_f16((float)x);
              }
      }
    };
    std::vector<std::thread> th;
    for (int t = 1; t < n_threads; ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
  }
  (void)vbase;
  tb.n_blocks += nb;
}

}  // namespace tlt
