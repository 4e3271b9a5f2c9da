// Rendering through the spatially compressed transport -- Eq. (10); Steps 2,
// 4 and 5 of Sec. 4.
//
//   y[c, u]       = sum_{(k, j) in row u} g_k[c] Z_k[u, j] Ehat[j, c]   (k_sp_rows)
//   B[perm[o], c] = sum_u S[o, u] y[c, u],  S = w_1^{-1}                (k_sp_synth)
//
// Z is a CSR over the output coefficient u (column word (k << 24) | j).  Work
// items bound the entries one lane group streams: a long row is cut into
// several consecutive items.  Every item writes its partial sums, and Step 5
// reads y[c, u] as the sum of row u's items -- no atomics, no buffer to
// clear, nothing shared between workgroups within a launch.
//
// k_sp_rows has two forms.  For up to 16 output columns a group of 16, 32 or
// 64 lanes takes one item: each lane loads a batch of its own entries
// (column word, value, and the short Ehat row it points at) before using
// any, and the group sums its lanes at the end.  For more columns the lanes
// split the columns: each entry is broadcast from the lane that loaded it
// and every lane reads its own column of that Ehat row.
//
// Step 5 is the CDF 9/7 synthesis as a fixed sparse matrix (a few tens of
// entries per output position, built on the host by synthesising every unit
// coefficient), expanded at load over the work items of each coefficient's
// row: B[o] = sum over (item, weight) of weight * partial[item].  A group of
// lanes per output position loads its entries (contiguous), gathers the
// partials and sums across the group.

#include "device_common.h"
#include "spatial.h"

namespace tlt {

namespace {

constexpr int SP_WIDE_ITEMS = 4;            // wide form: one item per wave, 256 threads

template <typename CT, int NC, int G, int U>
__global__ __launch_bounds__(256) void k_sp_rows(SpatialArgs a) {
  __shared__ CT gs[SP_MAX_K * NC];
  const CT *gcol = (const CT *)a.gcol;
  for (int i = threadIdx.x; i < a.K * NC; i += 256) {
    const int k = i / NC, c = i - k * NC;
    gs[i] = c < a.C ? gcol[(size_t)k * a.Cs + c] : CT(0);
  }
  __syncthreads();
  // G lanes per item, 256 / G items per workgroup; groups are aligned in the
  // wave, so a group exits or stays as a whole
  const int sub = threadIdx.x & (G - 1);
  const int item = blockIdx.x * (256 / G) + threadIdx.x / G;
  if (item >= a.n_items) return;
  const int64_t e0 = a.item_e0[item], e1 = a.item_e1[item];
  const uint32_t *col = a.col;
  const CT *val = (const CT *)a.val;
  const CT *ehat = (const CT *)a.ehat;
  CT acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0;
  for (int64_t base = e0; base < e1; base += G * U) {
    uint32_t cw[U];
    CT v[U];
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const int64_t e = base + r * G + sub;
      const bool ok = e < e1;
      cw[r] = col[ok ? e : e0];
      v[r] = ok ? val[e] : CT(0);
    }
    CT er[U][NC];
#pragma unroll
    for (int r = 0; r < U; ++r)
      RowLoad<CT, NC>::load(ehat + (size_t)(cw[r] & 0xffffffu) * a.Cs, er[r]);
#pragma unroll
    for (int r = 0; r < U; ++r) {
      const CT *g = gs + (cw[r] >> 24) * NC;
#pragma unroll
      for (int c = 0; c < NC; ++c) acc[c] = fma(v[r] * g[c], er[r][c], acc[c]);
    }
  }
  CT mine = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    CT t = acc[c];
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) t += __shfl_xor(t, m, 64);
    if (sub == c) mine = t;
  }
  if (sub < a.C) ((CT *)a.part)[(size_t)item * a.C + sub] = mine;
}

template <typename CT>
__global__ __launch_bounds__(256) void k_sp_rows_wide(SpatialArgs a) {
  extern __shared__ __align__(16) unsigned char raw[];
  CT *gs = reinterpret_cast<CT *>(raw);               // [K][64] of this column group
  const int c0 = blockIdx.y * 64;
  const CT *gcol = (const CT *)a.gcol;
  for (int i = threadIdx.x; i < a.K * 64; i += 256) {
    const int k = i >> 6, c = c0 + (i & 63);
    gs[i] = c < a.C ? gcol[(size_t)k * a.Cs + c] : CT(0);
  }
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int item = blockIdx.x * SP_WIDE_ITEMS + (threadIdx.x >> 6);
  if (item >= a.n_items) return;
  const int64_t e0 = a.item_e0[item], e1 = a.item_e1[item];
  const int c = c0 + lane;
  const int cc = c < a.Cs ? c : a.Cs - 1;             // stays inside the Ehat row
  const CT *ehat = (const CT *)a.ehat;
  const CT *val = (const CT *)a.val;
  CT acc = 0;
  for (int64_t base = e0; base < e1; base += 64) {
    const int64_t e = base + lane;
    const bool ok = e < e1;
    const uint32_t cw = a.col[ok ? e : e0];
    const CT v = ok ? val[e] : CT(0);
    const int n = (int)min<int64_t>(64, e1 - base);
    for (int t = 0; t < n; ++t) {
      const uint32_t w = (uint32_t)__shfl((int)cw, t, 64);
      const CT vt = __shfl(v, t, 64);
      acc = fma(vt * gs[(w >> 24) * 64 + lane], ehat[(size_t)(w & 0xffffffu) * a.Cs + cc], acc);
    }
  }
  if (c < a.C) ((CT *)a.part)[(size_t)item * a.C + c] = acc;
}

// B[q][perm[o]][ch] for the NC columns c0 .. c0+NC-1 (c = 3q + ch): G lanes
// per output position, each loading E of its (item, weight) entries before
// gathering the items' partial sums
template <typename CT, int NC, int G, int E>
__global__ __launch_bounds__(256) void k_sp_synth(SpatialArgs a) {
  const int sub = threadIdx.x & (G - 1);
  const int o = blockIdx.x * (256 / G) + threadIdx.x / G;
  if (o >= a.N) return;
  const int c0 = blockIdx.y * NC;
  const CT *part = (const CT *)a.part + c0;
  const CT *sw = (const CT *)a.syn_w + (size_t)o * a.syn_len;
  const int32_t *sc = a.syn_col + (size_t)o * a.syn_len;
  CT acc[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) acc[c] = 0;
  for (int t0 = 0; t0 < a.syn_len; t0 += G * E) {
    int it[E];
    CT w[E];
#pragma unroll
    for (int r = 0; r < E; ++r) {
      it[r] = sc[t0 + r * G + sub];
      w[r] = sw[t0 + r * G + sub];
    }
#pragma unroll
    for (int r = 0; r < E; ++r) {
      const CT *p = part + (size_t)it[r] * a.C;
#pragma unroll
      for (int c = 0; c < NC; ++c)
        if (c0 + c < a.C) acc[c] = fma(w[r], p[c], acc[c]);
    }
  }
  CT mine = 0;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    CT t = acc[c];
#pragma unroll
    for (int m = G / 2; m >= 1; m >>= 1) t += __shfl_xor(t, m, 64);
    if (sub == c) mine = t;
  }
  if (sub < NC && c0 + sub < a.C) {
    const int cg = c0 + sub, q = cg / 3, ch = cg - 3 * q;
    ((CT *)a.B)[((int64_t)q * a.N + a.perm[o]) * 3 + ch] = mine;
  }
}

template <typename CT, int NC, int G>
hipError_t rows_u(const SpatialArgs &a, hipStream_t st) {
  const unsigned nb = (unsigned)((a.n_items + 256 / G - 1) / (256 / G));
  // register budget: at most 64 Ehat values in flight per lane
  constexpr int U16 = NC <= 4 ? 16 : (NC <= 8 ? 8 : 4);
  constexpr int U8 = NC <= 8 ? 8 : 4;
  if (a.unroll >= 16)
    TLT_LAUNCH((k_sp_rows<CT, NC, G, U16>), dim3(nb), dim3(256), 0, st, a);
  else if (a.unroll >= 8)
    TLT_LAUNCH((k_sp_rows<CT, NC, G, U8>), dim3(nb), dim3(256), 0, st, a);
  else
    TLT_LAUNCH((k_sp_rows<CT, NC, G, 4>), dim3(nb), dim3(256), 0, st, a);
  return hipGetLastError();
}

template <typename CT, int NC>
hipError_t rows_narrow(const SpatialArgs &a, hipStream_t st) {
  switch (a.lanes_per_item) {
    case 16: return rows_u<CT, NC, 16>(a, st);
    case 32: return rows_u<CT, NC, 32>(a, st);
    default: return rows_u<CT, NC, 64>(a, st);
  }
}

template <typename CT>
hipError_t rows_go(const SpatialArgs &a, hipStream_t st) {
  if (a.n_items == 0) return hipSuccess;
  if (a.C <= 4) return rows_narrow<CT, 4>(a, st);
  if (a.C <= 8) return rows_narrow<CT, 8>(a, st);
  if (a.C <= 16) return rows_narrow<CT, 16>(a, st);
  const unsigned nb = (unsigned)((a.n_items + SP_WIDE_ITEMS - 1) / SP_WIDE_ITEMS);
  TLT_LAUNCH((k_sp_rows_wide<CT>), dim3(nb, (a.C + 63) / 64), dim3(256),
             sizeof(CT) * 64 * (size_t)a.K, st, a);
  return hipGetLastError();
}

template <typename CT, int NC, int G>
hipError_t synth_g(const SpatialArgs &a, hipStream_t st) {
  const unsigned nb = (unsigned)((a.N + 256 / G - 1) / (256 / G));
  const dim3 grid(nb, (a.C + NC - 1) / NC);
  // entries per lane and pass: syn_len / G when it is at most 8, else 4 or
  // 8 per pass (syn_len is a multiple of G, and of 4 G beyond 8 G)
  switch (a.syn_len / G) {
    case 1: TLT_LAUNCH((k_sp_synth<CT, NC, G, 1>), grid, dim3(256), 0, st, a); break;
    case 2: TLT_LAUNCH((k_sp_synth<CT, NC, G, 2>), grid, dim3(256), 0, st, a); break;
    case 3: TLT_LAUNCH((k_sp_synth<CT, NC, G, 3>), grid, dim3(256), 0, st, a); break;
    case 4: TLT_LAUNCH((k_sp_synth<CT, NC, G, 4>), grid, dim3(256), 0, st, a); break;
    case 5: TLT_LAUNCH((k_sp_synth<CT, NC, G, 5>), grid, dim3(256), 0, st, a); break;
    case 6: TLT_LAUNCH((k_sp_synth<CT, NC, G, 6>), grid, dim3(256), 0, st, a); break;
    case 7: TLT_LAUNCH((k_sp_synth<CT, NC, G, 7>), grid, dim3(256), 0, st, a); break;
    case 8: TLT_LAUNCH((k_sp_synth<CT, NC, G, 8>), grid, dim3(256), 0, st, a); break;
    default:
      if ((a.syn_len / G) % 8 == 0)
        TLT_LAUNCH((k_sp_synth<CT, NC, G, 8>), grid, dim3(256), 0, st, a);
      else
        TLT_LAUNCH((k_sp_synth<CT, NC, G, 4>), grid, dim3(256), 0, st, a);
  }
  return hipGetLastError();
}

template <typename CT, int NC>
hipError_t synth_nc(const SpatialArgs &a, hipStream_t st) {
  switch (a.syn_lanes) {
    case 8: return synth_g<CT, NC, 8>(a, st);
    case 16: return synth_g<CT, NC, 16>(a, st);
    default: return synth_g<CT, NC, 32>(a, st);
  }
}

template <typename CT>
hipError_t synth_go(const SpatialArgs &a, hipStream_t st) {
  if (a.C <= 4) return synth_nc<CT, 4>(a, st);
  return synth_nc<CT, 8>(a, st);          // column groups of 8 over grid y
}

bool args_ok(const SpatialArgs &a) {
  return a.K >= 1 && a.K <= SP_MAX_K && a.N >= 8 && a.C >= 1 && a.C <= a.Cs &&
         !(a.C <= 16 && a.Cs < 16) && a.syn_len >= 1 && a.syn_len % a.syn_lanes == 0 &&
         (a.syn_len <= 8 * a.syn_lanes || a.syn_len % (4 * a.syn_lanes) == 0) &&
         (a.lanes_per_item == 16 || a.lanes_per_item == 32 || a.lanes_per_item == 64) &&
         (a.syn_lanes == 8 || a.syn_lanes == 16 || a.syn_lanes == 32);
}

}  // namespace

hipError_t launch_spatial_rows(const SpatialArgs &a, bool fp64, hipStream_t st) {
  if (!args_ok(a)) return hipErrorInvalidValue;
  return fp64 ? rows_go<double>(a, st) : rows_go<float>(a, st);
}

hipError_t launch_spatial_synthesis(const SpatialArgs &a, bool fp64, hipStream_t st) {
  if (!args_ok(a)) return hipErrorInvalidValue;
  return fp64 ? synth_go<double>(a, st) : synth_go<float>(a, st);
}

}  // namespace tlt
