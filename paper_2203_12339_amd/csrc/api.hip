// C ABI of libtlt.so: context, transport loading, per-frame render and its
// adjoint.  See include/tlt.h for the contract of every entry point.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/tlt.h"
#include "host_internal.h"
#include "kernels.h"
#include "spatial.h"

using namespace tlt;

namespace tlt {
StageEvents &stage_events() {
  static thread_local StageEvents ev;
  return ev;
}
}  // namespace tlt

// Scratch of render_backward_noalloc: the adjoint's partial rows and group
// sums in a file-scope device array, so that the call allocates nothing.
// Each GPU the library runs on holds its own copy until the process ends.
// In host code the name `scratch` is only a host-side stand-in: host code
// uses the device address hipGetSymbolAddress returns for the current
// device, looked up once per device by tlt_create (scratch_addr below).
static __device__ __align__(256) unsigned char scratch[TLT_NOALLOC_SCRATCH_BYTES];

namespace {
std::mutex scratch_mu;
std::vector<void *> scratch_addr;   // per device index; null until looked up
}  // namespace

struct tlt_ctx {
  int device = 0;
  std::string err;

  // transport
  bool loaded = false;
  bool bf16_plain = false;   // BF16 storage without residual words in the tiles
  int N = 0, n_pad = 0, n_sh = 0, n_shp = 0, K = 0, nr = 0, wavelet = 0, vdt = 0, tdt = 0;
  int64_t n_keep = 0;
  int n_rows = 0;  // rows of Ehat: n_pad (Haar) or N (plain)
  bool fp64 = false;
  size_t esz = 4;
  int32_t *col = nullptr;
  void *val = nullptr;
  void *T = nullptr;
  void *area = nullptr;
  int32_t *perm = nullptr;
  double *rn = nullptr, *basis = nullptr;
  double mat_range[6] = {0, 0, 0, 0, 0, 0};
  bool has_range = false;

  // G = H pad(A o T) [n_rows][G_ld] (column lm: Haar of the area-weighted
  // transfer column), so that Ehat = G L with no per-frame Haar levels
  void *Gmat = nullptr, *Gpart = nullptr;
  int G_ld = 0;
  int tune_irr_haar = 0;   // 1: per-frame Haar of A o (T L) instead of G L
  int tune_head_off = 0;   // 1: no residual words for the coarsest BF16 columns
  // device build of BF16 tiles: residuals of the coarsest columns
  // [N*K][head_cols] (during load_transport only) and their count
  uint16_t *build_res = nullptr;
  int head_cols = 0;

  // lighting-transfer product P[k][v][Psh] = W_k G, rows in original vertex
  // order (folded lighting and the adjoint)
  bool have_P = false;
  int Psh = 0, Gs = 0;
  void *P = nullptr;
  // FP16 copy of P (16-bit storage, folded lighting; built at the first
  // folded render): sp P in matrix fragment order, p16_inv = 1 / sp
  void *P16 = nullptr;
  float p16_inv = 0.f;
  int tune_fold_fp32 = 0;   // 1: folded lighting on the float32 P

  // view for the outgoing Fresnel factor (set_view): cos(w_o, n) per
  // Morton position, compute precision
  void *view_cos = nullptr;
  bool view = false;

  // inputs of the next render
  const void *sh = nullptr;
  const void *E = nullptr;   // supplied irradiance (set_irradiance) instead of SH lighting
  bool use_E = false;
  int n_light = 0;
  const double *theta = nullptr;
  int n_mat = 0;
  // material validation flags written by the weights kernel (see PrepArgs):
  // pinned, coherent host memory, read by tlt_material_status
  int *mstat = nullptr, *mstat_dev = nullptr;
  bool mat_dirty = true, light_dirty = true;

  // column-dependent buffers
  int C = 0, Cs = 0, cpl = 0, n_out = 0, tile_req = 0;
  int buf_nlight = -1, buf_nmat = -1;
  void *Lm = nullptr, *ehat = nullptr, *partial = nullptr, *gcol = nullptr, *V = nullptr;
  void *ehat2 = nullptr;  // hi|lo split of Ehat for 16-bit tiles
  double *g64 = nullptr, *dg64 = nullptr;
  void *adj = nullptr;
  size_t adj_bytes = 0;
  void *fold = nullptr;   // folded lighting weights [K*Psh][Cs]
  size_t fold_bytes = 0;
  bool v_valid = false;   // V holds v_k of the current lighting (TLT_KEEP_TERMS)
  bool bwd_valid = false; // the last render was made with TLT_SAVE_FOR_BACKWARD
  void *scratch_dev = nullptr;   // this device's copy of the static adjoint scratch
  int n_chunks = 0, ch_rows = 0;

  // fragment-sparse tiles (see tlt.h): entry and fragment offsets, entry
  // columns, per-step m-tile masks, stored fragments
  bool tiles = false;
  int tV = 0, tR = 0, t_blocks = 0, t_max_union = 0;
  int64_t *t_off = nullptr, *t_foff = nullptr;
  int32_t *t_ucol = nullptr;
  uint16_t *t_mask = nullptr;
  void *t_val = nullptr;
  size_t t_val_bytes = 0;
  int64_t t_frags = 0;   // stored fragments
  bool t_sparse = false;     // fragment-sparse tiles (rows (k, o), step masks)
  int tune_tile_sparse = 0;  // 0 built-in, 1 dense, 2 fragment-sparse

  // spatially compressed transport (load_spatial): CSR of the kept entries
  // of Z_k = w_1 W_k^S over u, as work items of at most 2048 entries
  bool spatial = false;
  int sp_levels = 0, sp_sizes[32] = {0};
  int64_t sp_nnz = 0;
  std::vector<int64_t> sp_rowptr, sp_nnz_k;
  std::vector<double> sp_energy;
  uint32_t *sp_col = nullptr;
  void *sp_val = nullptr;
  int sp_items = 0;
  int64_t *sp_item_e = nullptr;   // [2][n_items]: first and one-past-last entry
  int sp_syn_len = 0, sp_syn_lanes = 16;   // w_1^{-1} over items, padded CSR [N][syn_len]
  int32_t *sp_syn_col = nullptr;
  void *sp_syn_w = nullptr;
  void *sp_part = nullptr;        // [n_items][C] partial sums
  size_t sp_part_bytes = 0;
  double sp_mean_item = 0.0;      // mean entries per item
  // launch tuning (tlt_set_tuning; 0 = built-in choice)
  int tune_sp_lanes = 0, tune_sp_unroll = 0, tune_sp_syn_lanes = 0, tune_sp_segment = 0;

  // tuning (tlt_set_tuning; 0 = built-in choice)
  int tune_tile_chunk = 0, tune_waves_per_cu = 0, tune_stream_epl = 0, tune_stream_nt = 0;
  int tune_tile_shape = 0;

  // transport partition: n_waves equal row ranges of part_rows = N*K rows;
  // split vertices cleared
  int n_waves = 0;
  int64_t part_rows = 0;
  int32_t *zero_v = nullptr;
  int n_zero = 0;

  // per-stage event timing
  bool prof = false;
  struct Ev { int stage; hipEvent_t a, b; };
  std::vector<Ev> pending;
  std::vector<hipEvent_t> pool;
  double prof_ms[6] = {0, 0, 0, 0, 0, 0};
  int64_t prof_n[6] = {0, 0, 0, 0, 0, 0};
};

namespace {

tlt_status hip_fail(tlt_ctx *c, hipError_t e, const char *what) {
  return fail(c ? &c->err : nullptr, TLT_E_HIP,
              std::string(what) + ": " + hipGetErrorString(e));
}

#define HIPC(ctx, expr)                                   \
  do {                                                    \
    hipError_t _e = (expr);                               \
    if (_e != hipSuccess) return hip_fail(ctx, _e, #expr); \
  } while (0)

template <typename T> void dfree(T *&p) {
  if (p) (void)hipFree((void *)p);
  p = nullptr;
}

tlt_status dalloc(tlt_ctx *c, void **p, size_t bytes, const char *what) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return fail(&c->err, e == hipErrorOutOfMemory ? TLT_E_OOM : TLT_E_HIP,
                std::string("allocating ") + what + " (" + std::to_string(bytes) +
                    " bytes): " + hipGetErrorString(e));
  }
  return TLT_OK;
}

size_t dtype_size(int dt) { return dt == TLT_F64 ? 8 : dt == TLT_F32 ? 4 : 2; }

int round_up(int x, int m) { return (x + m - 1) / m * m; }

const int kCpl[] = {4, 8, 12, 16, 24, 28, 32, 36, 48, 64};

int auto_cpl(int C) {
  for (int v : kCpl)
    if (v >= C) return v;
  return 48;
}

void free_columns(tlt_ctx *c) {
  dfree(c->Lm);
  dfree(c->ehat);
  dfree(c->ehat2);
  dfree(c->partial);
  dfree(c->gcol);
  dfree(c->V);
  dfree(c->g64);
  dfree(c->dg64);
  dfree(c->adj);
  c->adj_bytes = 0;
  dfree(c->fold);
  c->fold_bytes = 0;
  dfree(c->sp_part);
  c->sp_part_bytes = 0;
  c->C = c->Cs = c->n_out = 0;
  c->buf_nlight = c->buf_nmat = -1;
  c->v_valid = false;
  c->bwd_valid = false;
}

void free_spatial(tlt_ctx *c) {
  dfree(c->sp_col);
  dfree(c->sp_val);
  dfree(c->sp_item_e);
  dfree(c->sp_syn_col);
  dfree(c->sp_syn_w);
  dfree(c->sp_part);
  c->sp_part_bytes = 0;
  c->sp_syn_len = 0;
  c->sp_rowptr.clear();
  c->sp_nnz_k.clear();
  c->sp_energy.clear();
  c->sp_items = 0;
  c->sp_nnz = 0;
  c->sp_levels = 0;
  c->spatial = false;
}

void free_all(tlt_ctx *c) {
  dfree(c->build_res);
  c->build_res = nullptr;
  free_columns(c);
  free_spatial(c);
  dfree(c->view_cos);
  c->view = false;
  dfree(c->Gmat);
  dfree(c->Gpart);
  c->G_ld = 0;
  dfree(c->col);
  dfree(c->val);
  dfree(c->T);
  dfree(c->area);
  dfree(c->perm);
  dfree(c->rn);
  dfree(c->basis);
  dfree(c->P);
  dfree(c->P16);
  c->p16_inv = 0.f;
  dfree(c->zero_v);
  c->n_zero = 0;
  c->n_waves = 0;   // the partition belongs to the freed transport
  c->part_rows = 0;
  dfree(c->t_off);
  dfree(c->t_foff);
  dfree(c->t_ucol);
  dfree(c->t_mask);
  dfree(c->t_val);
  c->t_frags = 0;
  c->tiles = false;
  c->t_blocks = 0;
  c->have_P = false;
  c->loaded = false;
  c->sh = nullptr;
  c->theta = nullptr;
  c->n_light = c->n_mat = 0;
}

// Rows of Ehat per irradiance workgroup: 256, or 64 for Haar transforms
// whose 256-row chunks would give too few workgroups to fill the chip.
int prep_rows(const tlt_ctx *c, int Cs) {
  int r = std::min(c->n_rows, 256);
  if (c->wavelet == TLT_WAVELET_HAAR && (c->n_rows / 256) * (Cs / 16) < 512) r = std::min(c->n_rows, 64);
  return r;
}

// (Re)allocates every buffer whose size depends on the column count.
tlt_status ensure_columns(tlt_ctx *c) {
  const int n_out = std::max(c->n_light, c->n_mat);
  int cpl = c->tile_req ? c->tile_req : auto_cpl(3 * n_out);
  if (c->buf_nlight == c->n_light && c->buf_nmat == c->n_mat && cpl == c->cpl && c->ehat)
    return TLT_OK;
  free_columns(c);
  c->n_out = n_out;
  c->C = 3 * n_out;
  c->cpl = cpl;
  const int chunks = (c->C + cpl - 1) / cpl;
  c->Cs = round_up(std::max(c->C, chunks * cpl), 16);
  const size_t e = c->esz;
  tlt_status s;
  if ((s = dalloc(c, &c->Lm, e * c->n_shp * c->Cs, "lighting matrix")) != TLT_OK) return s;
  if ((s = dalloc(c, &c->ehat, e * (size_t)c->n_rows * c->Cs, "Ehat")) != TLT_OK) return s;
  if (c->tiles && c->vdt != TLT_F32 &&
      (s = dalloc(c, &c->ehat2, 4 * (size_t)c->n_rows * c->Cs, "Ehat split")) != TLT_OK)
    return s;
  const int ch_rows = prep_rows(c, c->Cs);
  const int n_chunks = (c->n_rows + ch_rows - 1) / ch_rows;
  if ((s = dalloc(c, &c->partial, e * (size_t)n_chunks * c->Cs, "Haar partials")) != TLT_OK) return s;
  if ((s = dalloc(c, &c->gcol, e * (size_t)c->K * c->Cs, "column weights")) != TLT_OK) return s;
  HIPC(c, hipMemset(c->gcol, 0, e * (size_t)c->K * c->Cs));
  if ((s = dalloc(c, (void **)&c->g64, sizeof(double) * c->n_mat * 3 * c->K, "g")) != TLT_OK) return s;
  if ((s = dalloc(c, (void **)&c->dg64, sizeof(double) * c->n_mat * 9 * c->K, "dg")) != TLT_OK) return s;
  c->ch_rows = ch_rows;
  c->n_chunks = n_chunks;
  c->buf_nlight = c->n_light;
  c->buf_nmat = c->n_mat;
  c->mat_dirty = c->light_dirty = true;
  return TLT_OK;
}

PrepArgs prep_args(tlt_ctx *c, int Cs, Cols cols) {
  PrepArgs a;
  std::memset(&a, 0, sizeof(a));
  a.fp64 = c->fp64;
  a.tdt = c->tdt;
  a.Cs = Cs;
  a.cols = cols;
  a.rn = c->rn;
  a.basis = c->basis;
  a.nr = c->nr;
  a.K = c->K;
  a.gk_stage = (size_t)c->K * c->nr <= 4096;   // 32 KB of basis in LDS
  a.mstat = c->mstat_dev;
  a.has_range = c->has_range;
  for (int p = 0; p < 3; ++p) {
    a.mat_lo[p] = c->mat_range[2 * p];
    a.mat_hi[p] = c->mat_range[2 * p + 1];
  }
  a.T = c->T;
  a.N = c->N;
  a.n_sh = c->n_sh;
  a.n_shp = c->n_shp;
  a.area = c->area;
  a.haar = c->wavelet == TLT_WAVELET_HAAR;
  a.n_rows = c->n_rows;
  a.ch_rows = prep_rows(c, Cs);
  a.n_chunks = (c->n_rows + a.ch_rows - 1) / a.ch_rows;
  return a;
}

// Equal row ranges per wave; vertices straddling two ranges are listed so
// the prep launch can clear their outputs before the atomic completion.
tlt_status ensure_partition(tlt_ctx *c) {
  const int wpc = c->tune_waves_per_cu > 0 ? c->tune_waves_per_cu : 32;
  const int nw = stream_waves(c->N, c->K, wpc);
  const int64_t R = (int64_t)c->N * c->K;
  if (nw == c->n_waves && R == c->part_rows) return TLT_OK;
  dfree(c->zero_v);
  c->n_zero = 0;
  c->n_waves = 0;
  c->part_rows = 0;
  const int64_t q = R / nw, rem = R % nw;
  std::vector<int32_t> z;
  for (int64_t w = 1; w < nw; ++w) {
    const int64_t r0 = w * q + std::min<int64_t>(w, rem);
    if (r0 % c->K) z.push_back((int32_t)(r0 / c->K));  // Morton position
  }
  if (!z.empty()) {
    std::vector<int32_t> hp(c->N);
    HIPC(c, hipMemcpy(hp.data(), c->perm, sizeof(int32_t) * c->N, hipMemcpyDeviceToHost));
    for (auto &v : z) v = hp[v];                         // original vertex id
    tlt_status s = dalloc(c, (void **)&c->zero_v, sizeof(int32_t) * z.size(), "split vertices");
    if (s != TLT_OK) return s;
    HIPC(c, hipMemcpy(c->zero_v, z.data(), sizeof(int32_t) * z.size(), hipMemcpyHostToDevice));
    c->n_zero = (int)z.size();
  }
  c->n_waves = nw;
  c->part_rows = R;
  return TLT_OK;
}

StreamArgs stream_args(tlt_ctx *c, const void *ehat, int Cs, int C, const void *gcol, void *B,
                       void *vsave, int vs_stride) {
  StreamArgs a;
  std::memset(&a, 0, sizeof(a));
  a.col = c->col;
  a.val = c->val;
  a.n_keep = (int)c->n_keep;
  a.K = c->K;
  a.N = c->N;
  a.ehat = ehat;
  a.Cs = Cs;
  a.C = C;
  a.gcol = gcol;
  a.perm = c->perm;
  a.B = B;
  a.vsave = vsave;
  a.vs_stride = vs_stride;
  a.R = (int64_t)c->N * c->K;
  a.n_waves = c->n_waves;
  a.epl = c->tune_stream_epl;
  a.nt = c->tune_stream_nt;
  return a;
}

TileArgs tile_args(tlt_ctx *c, const void *ehat, const void *ehat2, int Cs, int C,
                   const void *gcol, void *B, void *vsave, int vs_stride) {
  TileArgs a;
  std::memset(&a, 0, sizeof(a));
  a.blk_off = c->t_off;
  a.ucol = c->t_ucol;
  a.fmask = c->t_mask;
  a.foff = c->t_foff;
  a.val = c->t_val;
  a.V = c->tV;
  a.K = c->K;
  a.R = c->tR;
  a.n_blocks = c->t_blocks;
  a.max_union = c->t_max_union;
  a.N = c->N;
  a.ehat = ehat;
  a.ehat2 = ehat2;
  a.Cs = Cs;
  a.C = C;
  a.gcol = gcol;
  a.perm = c->perm;
  a.B = B;
  a.vsave = vsave;
  a.vs_stride = vs_stride;
  a.kc = c->tune_tile_chunk;
  a.shape = c->tune_tile_shape;
  a.stream_w = c->t_val_bytes > ((size_t)256 << 20);   // MI355X Infinity Cache: 256 MB
  a.sparse = c->t_sparse;
  return a;
}

// Vertices per tile block.  float32 storage streams the most bytes per
// kept coefficient, so it takes the smallest block (48..64 rows): nearby
// vertices share more of their kept columns, fewer stored zeros (measured
// ~10% fewer bytes at 48 than at 96 rows).  16-bit storage is bound by the
// staging of Ehat as well, so it takes the largest block (up to 128 rows),
// which shares each staged row among the most transport rows.
int auto_tile_vertices(int K, int vdt) {
  if (vdt == TLT_F32)
    for (int R = 48; R <= 64; R += 16)
      if (R % K == 0) return R / K;
  for (int V : {32, 16, 8, 4, 64})
    if (V * K >= 64 && V * K <= 128 && (V * K) % 16 == 0) return V;
  return 0;
}

tlt_status ensure_V(tlt_ctx *c) {
  if (c->V) return TLT_OK;
  return dalloc(c, &c->V, c->esz * (size_t)c->K * c->N * c->Cs, "saved v_k");
}

// G = Haar(pad(A o T)) and P = W G (per k), for the lighting gradient.
// Builds G = H pad(A o T) once: the irradiance pass with identity lighting.
tlt_status ensure_G(tlt_ctx *c, hipStream_t st) {
  if (c->Gmat) return TLT_OK;
  const int ld = round_up(c->n_sh, 16);
  Cols ident{c->n_sh, 1, 1, 1};
  PrepArgs a = prep_args(c, ld, ident);
  tlt_status s;
  if ((s = dalloc(c, &c->Gpart, c->esz * (size_t)a.n_chunks * ld, "G partials")) != TLT_OK) return s;
  if ((s = dalloc(c, &c->Gmat, c->esz * (size_t)c->n_rows * ld, "G")) != TLT_OK) {
    dfree(c->Gpart);
    return s;
  }
  a.n_tl_blocks = a.n_chunks * (ld / 16);
  a.sh = nullptr;
  a.ehat = c->Gmat;
  a.partial = c->Gpart;
  a.ehat2 = nullptr;
  const hipError_t he = launch_prep(a, st);
  if (he != hipSuccess) {
    dfree(c->Gmat);
    dfree(c->Gpart);
    return hip_fail(c, he, "building G = H (A o T)");
  }
  c->G_ld = ld;
  return TLT_OK;
}

tlt_status ensure_P(tlt_ctx *c, hipStream_t st) {
  if (c->have_P) return TLT_OK;
  int cplP = 0;
  for (int v : kCpl)
    if (v >= c->n_sh) { cplP = v; break; }
  if (!cplP) return fail(&c->err, TLT_E_ARG, "n_sh too large for the adjoint");
  c->Psh = cplP;
  c->Gs = round_up(cplP, 16);
  const size_t e = c->esz;
  void *G = nullptr, *G2 = nullptr, *part = nullptr, *gz = nullptr;
  tlt_status s;
  Cols ident{c->Psh, 1, 1, 1};
  PrepArgs a = prep_args(c, c->Gs, ident);
  if ((s = dalloc(c, &c->P, e * (size_t)c->K * c->N * c->Psh, "P")) != TLT_OK) return s;
  if ((s = dalloc(c, &G, e * (size_t)c->n_rows * c->Gs, "G")) != TLT_OK) goto out;
  if ((s = dalloc(c, &part, e * (size_t)a.n_chunks * c->Gs, "G partials")) != TLT_OK) goto out;
  if ((s = dalloc(c, &gz, e * (size_t)c->K * c->Gs, "zero weights")) != TLT_OK) goto out;
  if (c->tiles && c->vdt != TLT_F32 &&
      (s = dalloc(c, &G2, 4 * (size_t)c->n_rows * c->Gs, "G split")) != TLT_OK)
    goto out;
  {
    a.n_tl_blocks = a.n_chunks * (c->Gs / 16);
    a.sh = nullptr;  // identity lighting: column lm of G is Haar(pad(A o T[:, lm]))
    a.ehat = G;
    a.partial = part;
    a.ehat2 = G2;
    a.split = c->vdt == TLT_BF16 ? 1 : 2;
    StreamArgs sa = stream_args(c, G, c->Gs, c->Psh, gz, nullptr, c->P, c->Psh);
    hipError_t he;
    if ((he = hipMemset(gz, 0, e * (size_t)c->K * c->Gs)) != hipSuccess ||
        (he = launch_prep(a, st)) != hipSuccess ||
        (he = c->tiles ? launch_tiles(tile_args(c, G, G2, c->Gs, c->Psh, nullptr, nullptr, c->P, c->Psh),
                                      c->vdt, st)
                       : launch_stream(sa, c->vdt, c->fp64, c->Psh, st)) != hipSuccess ||
        (he = hipStreamSynchronize(st)) != hipSuccess) {
      s = hip_fail(c, he, "building the lighting-transfer product");
      goto out;
    }
  }
  c->have_P = true;
  s = TLT_OK;
out:
  dfree(G);
  dfree(G2);
  dfree(part);
  dfree(gz);
  return s;
}

// The FP16 copy of P for the folded product (16-bit storage): scale sp puts
// the largest |P| in [2^13, 2^14).  A P that is not finite keeps the float32
// product (TLT_E_STATE otherwise would block a render the float32 form can
// do).
tlt_status ensure_P16(tlt_ctx *c, hipStream_t st) {
  if (c->P16 || c->vdt == TLT_F32 || c->fp64) return TLT_OK;
  const int J = c->K * c->Psh;
  if ((J + 31) / 32 > FOLD16_MAX_STEPS) return TLT_OK;
  unsigned *mx = nullptr;
  tlt_status s;
  if ((s = dalloc(c, (void **)&mx, sizeof(unsigned), "P maximum")) != TLT_OK) return s;
  unsigned bits = 0;
  hipError_t he;
  if ((he = hipMemset(mx, 0, sizeof(unsigned))) != hipSuccess ||
      (he = launch_fold_absmax((const float *)c->P, (int64_t)c->N * J, mx, st)) != hipSuccess ||
      (he = hipMemcpyAsync(&bits, mx, sizeof(unsigned), hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess) {
    dfree(mx);
    return hip_fail(c, he, "P maximum");
  }
  dfree(mx);
  float pmax;
  std::memcpy(&pmax, &bits, sizeof(pmax));
  if (!std::isfinite(pmax)) return TLT_OK;
  int e = 0;
  (void)std::frexp(pmax, &e);
  const float sp = pmax > 0.f ? std::ldexp(1.f, 14 - e) : 1.f;
  if ((s = dalloc(c, &c->P16, fold16_bytes(c->N, J), "P (FP16)")) != TLT_OK) return s;
  if ((he = launch_fold_pack((const float *)c->P, c->N, J, sp, c->P16, st)) != hipSuccess ||
      (he = hipStreamSynchronize(st)) != hipSuccess) {
    dfree(c->P16);
    return hip_fail(c, he, "P (FP16)");
  }
  c->p16_inv = 1.f / sp;
  return TLT_OK;
}

// Stage timer: hands an event pair to the launches of one stage (written by
// the kernel dispatches themselves) and queues the pair for reading.
struct StageTimer {
  tlt_ctx *c;
  int stage;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(tlt_ctx *c_, int stage_, hipStream_t st_) : c(c_), stage(stage_), st(st_) {
    if (!c->prof) return;
    a = take();
    b = take();
    if (a && b) stage_events() = StageEvents{a, b, 0};
  }
  hipEvent_t take() {
    if (!c->pool.empty()) {
      hipEvent_t e = c->pool.back();
      c->pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
  }
  ~StageTimer() {
    if (!c->prof) return;
    const int n = stage_events().launches;
    stage_events() = StageEvents{};
    if (!a || !b) return;
    if (n > 0) {
      c->pending.push_back({stage, a, b});
    } else {  // nothing launched: the pair was never written
      c->pool.push_back(a);
      c->pool.push_back(b);
    }
  }
};

void prof_drain(tlt_ctx *c) {
  for (auto &e : c->pending) {
    float ms = 0.f;
    if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      c->prof_ms[e.stage] += ms;
      c->prof_n[e.stage] += 1;
    }
    c->pool.push_back(e.a);
    c->pool.push_back(e.b);
  }
  c->pending.clear();
}

float half_to_float(uint16_t h) {
  const uint32_t sgn = (uint32_t)(h >> 15) << 31;
  const int ex = (h >> 10) & 31;
  uint32_t man = h & 1023;
  uint32_t bits;
  if (ex == 0) {
    if (man == 0) {
      bits = sgn;
    } else {  // subnormal: value = man * 2^-24
      float f = std::ldexp((float)man, -24);
      return (h >> 15) ? -f : f;
    }
  } else if (ex == 31) {
    bits = sgn | 0x7f800000u | (man << 13);
  } else {
    bits = sgn | ((uint32_t)(ex - 15 + 127) << 23) | (man << 13);
  }
  float f;
  std::memcpy(&f, &bits, 4);
  return f;
}

double widen(const void *p, int dt, size_t i) {
  switch (dt) {
    case TLT_F64: return ((const double *)p)[i];
    case TLT_F32: return ((const float *)p)[i];
    case TLT_BF16: {
      uint32_t b = (uint32_t)((const uint16_t *)p)[i] << 16;
      float f;
      std::memcpy(&f, &b, 4);
      return f;
    }
    default: return half_to_float(((const uint16_t *)p)[i]);
  }
}

}  // namespace

extern "C" {

const char *tlt_version(void) { return "tlt 0.1 gfx950"; }

tlt_status tlt_create(tlt_ctx **out, int hip_device) {
  if (!out) return fail(nullptr, TLT_E_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess || n <= 0)
    return fail(nullptr, TLT_E_HIP, std::string("no HIP device: ") + hipGetErrorString(e));
  if (hip_device < 0 || hip_device >= n) return fail(nullptr, TLT_E_ARG, "device index out of range");
  e = hipSetDevice(hip_device);
  if (e != hipSuccess) return fail(nullptr, TLT_E_HIP, hipGetErrorString(e));
  void *sp = nullptr;
  {
    // this device's copy of the static scratch, with the device current
    std::lock_guard<std::mutex> lock(scratch_mu);
    if ((int)scratch_addr.size() < n) scratch_addr.resize(n, nullptr);
    if (!scratch_addr[hip_device]) {
      e = hipGetSymbolAddress(&scratch_addr[hip_device], HIP_SYMBOL(scratch));
      if (e != hipSuccess) {
        scratch_addr[hip_device] = nullptr;
        return fail(nullptr, TLT_E_HIP, std::string("static scratch address: ") + hipGetErrorString(e));
      }
    }
    sp = scratch_addr[hip_device];
  }
  tlt_ctx *c = new (std::nothrow) tlt_ctx;
  if (!c) return fail(nullptr, TLT_E_OOM, "context allocation");
  c->device = hip_device;
  c->scratch_dev = sp;
  e = hipHostMalloc((void **)&c->mstat, 4 * sizeof(int), hipHostMallocMapped | hipHostMallocCoherent);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&c->mstat_dev, c->mstat, 0);
  if (e != hipSuccess) {
    if (c->mstat) (void)hipHostFree(c->mstat);
    delete c;
    return fail(nullptr, TLT_E_HIP, std::string("material status word: ") + hipGetErrorString(e));
  }
  for (int i = 0; i < 4; ++i) c->mstat[i] = 0;
  *out = c;
  return TLT_OK;
}

void tlt_destroy(tlt_ctx *c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  prof_drain(c);
  for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
  c->pool.clear();
  free_all(c);
  if (c->mstat) (void)hipHostFree(c->mstat);
  delete c;
}

const char *tlt_last_error(const tlt_ctx *c) {
  return c ? c->err.c_str() : g_thread_error.c_str();
}

tlt_status tlt_set_tile(tlt_ctx *c, int cpl) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (cpl != 0 && !stream_cpl_supported(cpl))
    return fail(&c->err, TLT_E_ARG, "unsupported columns_per_lane " + std::to_string(cpl));
  c->tile_req = cpl;
  return TLT_OK;
}

int tlt_get_tile(const tlt_ctx *c) { return c ? c->cpl : 0; }

// Transport rows built on the device from the Morton-ordered positions
// (kernel rows, Haar transform and exact top-n per row), in batches of
// vertices whose unsorted kept entries fit a bounded scratch buffer.
tlt_status device_build_rows(tlt_ctx *c, const tlt_transport_desc *d, int n_cols) {
  const int N = c->N, K = c->K, nr = c->nr;
  const int64_t n_keep = d->n_keep;
  const bool all = n_keep == n_cols;   // (limits checked with the description)
  const int chw = std::min(n_cols, build_chunk_columns());
  const int max_chunks = (n_cols + chw - 1) / chw;
  std::vector<double> slope((size_t)K * nr, 0.0);
  for (int k = 0; k < K; ++k)
    for (int m = 0; m + 1 < nr; ++m)
      slope[(size_t)k * nr + m] =
          (d->basis[(size_t)k * nr + m + 1] - d->basis[(size_t)k * nr + m]) / (d->r_nodes[m + 1] - d->r_nodes[m]);
  double *pos = nullptr, *dsl = nullptr, *sval = nullptr;
  int32_t *scol = nullptr;
  int *status = nullptr;
  tlt_status s = TLT_OK;
  hipError_t he = hipSuccess;
  const int64_t per_v = (int64_t)K * n_keep;
  const bool verbose = std::getenv("TLT_VERBOSE") != nullptr;
  const auto t0 = std::chrono::steady_clock::now();
  int64_t nvb = all ? N : std::max<int64_t>(1, ((int64_t)256 << 20) / (per_v * 12));
  nvb = std::min<int64_t>(nvb, N);
  if ((s = dalloc(c, (void **)&pos, sizeof(double) * 3 * (size_t)N, "positions")) != TLT_OK) goto out;
  if ((s = dalloc(c, (void **)&dsl, sizeof(double) * slope.size(), "slopes")) != TLT_OK) goto out;
  if ((s = dalloc(c, (void **)&status, sizeof(int), "build status")) != TLT_OK) goto out;
  if (!all) {
    if ((s = dalloc(c, (void **)&scol, sizeof(int32_t) * (size_t)(nvb * per_v), "build scratch")) != TLT_OK) goto out;
    if ((s = dalloc(c, (void **)&sval, sizeof(double) * (size_t)(nvb * per_v), "build scratch")) != TLT_OK) goto out;
  }
#define BTRY(x) if ((he = (x)) != hipSuccess) { s = hip_fail(c, he, #x); goto out; }
  BTRY(hipMemcpy(pos, d->position, sizeof(double) * 3 * (size_t)N, hipMemcpyHostToDevice));
  BTRY(hipMemcpy(dsl, slope.data(), sizeof(double) * slope.size(), hipMemcpyHostToDevice));
  BTRY(hipMemset(status, 0, sizeof(int)));
  for (int64_t o0 = 0; o0 < N; o0 += nvb) {
    if (verbose && o0 == 0) std::fprintf(stderr, "[tlt] building transport rows on the device\n");
    BuildArgs a{};
    a.pos = pos;
    a.rn = c->rn;
    a.basis = c->basis;
    a.slope = dsl;
    a.N = N;
    a.n_cols = n_cols;
    a.K = K;
    a.nr = nr;
    a.haar = c->wavelet == TLT_WAVELET_HAAR;
    a.hsq = 1.0 / std::sqrt(2.0);
    a.n_keep = n_keep;
    a.o0 = (int)o0;
    a.nv = (int)std::min<int64_t>(nvb, N - o0);
    a.all = all;
    a.max_chunks = max_chunks;
    a.scol = scol;
    a.sval = sval;
    a.col = c->col;
    a.val = c->val;
    a.vdt = c->vdt;
    a.status = status;
    a.res = c->build_res;
    a.head_cols = c->head_cols;
    for (int kg0 = 0; kg0 < K; kg0 += build_max_group()) {
      a.kg0 = kg0;
      BTRY(launch_build_select(a, std::min(build_max_group(), K - kg0), 0));
    }
    if (!all) BTRY(launch_build_sort(a, 0));
    if (verbose) {
      BTRY(hipDeviceSynchronize());
      std::fprintf(stderr, "[tlt] transport rows: %lld / %d vertices, %.1f s\n",
                   (long long)(o0 + a.nv), N,
                   std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count());
    }
  }
  BTRY(hipDeviceSynchronize());
  {
    int h = 0;
    BTRY(hipMemcpy(&h, status, sizeof(int), hipMemcpyDeviceToHost));
    if (h != 0) s = fail(&c->err, TLT_E_STATE, "device transport build failed its checks (" + std::to_string(h) + ")");
  }
#undef BTRY
out:
  dfree(pos);
  dfree(dsl);
  dfree(status);
  dfree(scol);
  dfree(sval);
  return s;
}

// Fragment-sparse tiles from the device rows: entry and fragment counts per
// block, offsets on the host, then entry ids, step masks and the stored
// fragments.
tlt_status device_build_tiles(tlt_ctx *c, int tV, int n_cols) {
  const int nb = (c->N + tV - 1) / tV;
  TileBuildArgs a{};
  a.col = c->col;
  a.val = c->val;
  a.esz = (int)dtype_size(c->vdt);
  a.N = c->N;
  a.K = c->K;
  a.V = tV;
  a.n_keep = c->n_keep;
  a.n_words = (n_cols + 31) / 32;
  a.n_blocks = nb;
  a.kstep = tile_kstep(c->vdt);
  a.res = c->build_res;
  a.head_cols = c->build_res ? c->head_cols : 0;
  // fragment-sparse tiles where they pay (measured): blocks of 256 rows of
  // 16-bit storage, whose W stream bounds the product; smaller blocks are
  // bound by their matrix work, which the sparse form cannot shorten (a
  // workgroup's waves wait for the fullest one at every staged chunk)
  {
    const bool want = c->vdt != TLT_F32 &&
                      (c->tune_tile_sparse == 2 || (c->tune_tile_sparse == 0 && tV * c->K == 256));
    a.order = want && tile_build_lds(a.n_words, true) <= (size_t)150 * 1024;
  }
  int64_t *cnt = nullptr, *fcnt = nullptr;
  size_t val_alloc = 0;
  tlt_status s = TLT_OK;
  hipError_t he = hipSuccess;
  const int kpl = a.kstep / 4;
  std::vector<int64_t> h(nb), hf(nb), ho(nb + 1, 0), fo(nb + 1, 0);
  if ((s = dalloc(c, (void **)&cnt, sizeof(int64_t) * nb, "tile counts")) != TLT_OK) return s;
  if ((s = dalloc(c, (void **)&fcnt, sizeof(int64_t) * nb, "tile fragment counts")) != TLT_OK) goto out;
#define BTRY(x) if ((he = (x)) != hipSuccess) { s = hip_fail(c, he, #x); goto out; }
  a.count = cnt;
  a.fcount = fcnt;
  BTRY(launch_tile_count(a, 0));
  BTRY(hipMemcpy(h.data(), cnt, sizeof(int64_t) * nb, hipMemcpyDeviceToHost));
  BTRY(hipMemcpy(hf.data(), fcnt, sizeof(int64_t) * nb, hipMemcpyDeviceToHost));
  c->t_max_union = 0;
  for (int b = 0; b < nb; ++b) {
    ho[b + 1] = ho[b] + h[b];
    fo[b + 1] = fo[b] + hf[b];
    c->t_max_union = std::max<int>(c->t_max_union, (int)h[b]);
    if (h[b] % a.kstep != 0 || hf[b] < 1 || hf[b] > h[b] / a.kstep * (tV * c->K / 16)) {
      s = fail(&c->err, TLT_E_STATE, "tile build: inconsistent entry or fragment count");
      goto out;
    }
  }
  c->tV = tV;
  c->tR = tV * c->K;
  c->t_blocks = nb;
  c->t_frags = fo[nb];
  c->t_sparse = a.order;
  c->t_val_bytes = (size_t)fo[nb] * 64 * kpl * a.esz;
  if ((s = dalloc(c, (void **)&c->t_off, sizeof(int64_t) * (nb + 1), "tile offsets")) != TLT_OK) goto out;
  if ((s = dalloc(c, (void **)&c->t_foff, sizeof(int64_t) * (nb + 1), "tile fragment offsets")) != TLT_OK) goto out;
  if ((s = dalloc(c, (void **)&c->t_ucol, sizeof(int32_t) * (size_t)ho[nb], "tile columns")) != TLT_OK) goto out;
  if ((s = dalloc(c, (void **)&c->t_mask, sizeof(uint16_t) * (size_t)(ho[nb] / a.kstep), "tile masks")) != TLT_OK) goto out;
  val_alloc = c->t_val_bytes;
  if ((s = dalloc(c, &c->t_val, val_alloc, "tile values")) != TLT_OK) goto out;
  BTRY(hipMemcpy(c->t_off, ho.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice));
  BTRY(hipMemcpy(c->t_foff, fo.data(), sizeof(int64_t) * (nb + 1), hipMemcpyHostToDevice));
  BTRY(hipMemset(c->t_val, 0, val_alloc));
  a.blk_off = c->t_off;
  a.frag_off = c->t_foff;
  a.ucol = c->t_ucol;
  a.mask = c->t_mask;
  a.tval = c->t_val;
  BTRY(launch_tile_fill(a, 0));
  BTRY(hipDeviceSynchronize());
  c->tiles = true;
#undef BTRY
out:
  dfree(cnt);
  dfree(fcnt);
  return s;
}

}  // extern "C"

namespace {

// Layout of the tiles a descriptor asks for: vertices per block (0 when
// tiles are not possible) and whether they are built.
struct TilePlan {
  int tV = 0;
  bool ok = false, want = false;
};

TilePlan tile_plan(const tlt_transport_desc *d, int n_cols) {
  TilePlan t;
  t.tV = d->tile_vertices > 0 ? d->tile_vertices : auto_tile_vertices(d->K, d->value_dtype);
  // (the tile build keeps two bitmaps of n_cols bits in LDS)
  t.ok = t.tV > 0 && t.tV * d->K >= 48 && t.tV * d->K <= tile_max_rows(d->value_dtype) &&
         (t.tV * d->K) % 16 == 0 &&
         (size_t)8 * ((n_cols + 31) / 32) <= (size_t)150 * 1024;
  t.want = d->value_dtype != TLT_F64 && d->layout != TLT_LAYOUT_ROWS && t.ok;
  return t;
}

// Every host-side check of a transport description, before any device
// work: sizes, dtypes, the permutation, the areas and (when given) the
// rows' columns.  TLT_E_ARG / TLT_E_FORMAT with a message in *err.
tlt_status check_transport_desc(const tlt_transport_desc *d, std::string *err) {
  if (!d) return fail(err, TLT_E_ARG, "NULL transport description");
  const int N = d->n_vertices;
  if (N < 1) return fail(err, TLT_E_ARG, "n_vertices must be >= 1");
  if (d->wavelet != TLT_WAVELET_NONE && d->wavelet != TLT_WAVELET_HAAR)
    return fail(err, TLT_E_ARG, "unknown wavelet");
  int n_pad = 1;
  while (n_pad < N) n_pad <<= 1;
  if (d->wavelet == TLT_WAVELET_HAAR && d->n_pad != n_pad)
    return fail(err, TLT_E_ARG, "n_pad must be the next power of two >= n_vertices");
  if (d->wavelet == TLT_WAVELET_HAAR && n_pad > (1 << 19))
    return fail(err, TLT_E_ARG, "n_pad above 2^19 is not supported");
  const int n_cols = d->wavelet == TLT_WAVELET_HAAR ? n_pad : N;
  if (d->n_sh < 1 || d->n_sh > 64) return fail(err, TLT_E_ARG, "n_sh must be in 1..64");
  if (d->K < 1 || d->K > 64) return fail(err, TLT_E_ARG, "K must be in 1..64");
  if (d->n_r < 2 || d->n_r > 1024) return fail(err, TLT_E_ARG, "n_r must be in 2..1024");
  if (d->n_keep < 1 || d->n_keep > n_cols) return fail(err, TLT_E_ARG, "n_keep out of range");
  for (int dt : {d->value_dtype, d->transfer_dtype})
    if (dt < TLT_F64 || dt > TLT_F16) return fail(err, TLT_E_ARG, "unknown dtype");
  if ((d->value_dtype == TLT_F64) != (d->transfer_dtype == TLT_F64))
    return fail(err, TLT_E_ARG, "transfer is F64 exactly when the transport is F64");
  if (d->layout < TLT_LAYOUT_AUTO || d->layout > TLT_LAYOUT_TILES) return fail(err, TLT_E_ARG, "unknown layout");
  if (d->tile_vertices < 0) return fail(err, TLT_E_ARG, "tile_vertices must be >= 0");
  if (d->val_is_f64 != 0 && d->val_is_f64 != 1) return fail(err, TLT_E_ARG, "val_is_f64 must be 0 or 1");
  if (d->val_is_f64 && !d->col) return fail(err, TLT_E_ARG, "val_is_f64 applies to rows given in col/val");
  if (!d->transfer || !d->area || !d->perm || !d->r_nodes || !d->basis)
    return fail(err, TLT_E_ARG, "NULL geometry array");
  if (!d->col && !d->position) return fail(err, TLT_E_ARG, "need col/val or position");
  if (d->col && !d->val) return fail(err, TLT_E_ARG, "col given without val");
  const TilePlan tp = tile_plan(d, n_cols);
  if (d->layout == TLT_LAYOUT_TILES && (d->value_dtype == TLT_F64 || !tp.ok))
    return fail(err, TLT_E_ARG,
                "tiles need non-F64 storage, 48 <= V*K <= 128 (256 for 16-bit storage), V*K % 16 == 0 "
                "and at most 614400 columns");
  if (!d->col) {
    // limits of the device build of the rows
    if (d->n_keep != n_cols && d->n_keep > build_sort_max())
      return fail(err, TLT_E_ARG,
                  "device build keeps at most " + std::to_string(build_sort_max()) +
                      " coefficients per row (or all); pass rows built on the host");
    if (n_cols > (1 << 20)) return fail(err, TLT_E_ARG, "device build supports at most 2^20 columns");
    if (d->wavelet == TLT_WAVELET_HAAR && n_cols < 8)
      return fail(err, TLT_E_ARG, "device build of Haar rows needs n_pad >= 8");
  }
  {
    std::vector<char> seen(N, 0);
    for (int i = 0; i < N; ++i) {
      const int p = d->perm[i];
      if (p < 0 || p >= N || seen[p]) return fail(err, TLT_E_FORMAT, "perm is not a permutation");
      seen[p] = 1;
    }
  }
  for (int i = 0; i < N; ++i)
    if (!(d->area[i] > 0.0) || !std::isfinite(d->area[i]))
      return fail(err, TLT_E_ARG, "areas must be positive and finite");
  if (d->col) {
    const int64_t n_rowsW = (int64_t)N * d->K;
    for (int64_t r = 0; r < n_rowsW; ++r) {
      const int32_t *cr = d->col + r * d->n_keep;
      for (int64_t e = 0; e < d->n_keep; ++e) {
        if (cr[e] < 0 || cr[e] >= n_cols)
          return fail(err, TLT_E_FORMAT, "column index out of range in row " + std::to_string(r));
        if (e > 0 && cr[e] <= cr[e - 1])
          return fail(err, TLT_E_FORMAT, "columns not ascending in row " + std::to_string(r));
      }
    }
  }
  return TLT_OK;
}

}  // namespace

extern "C" {

tlt_status tlt_check_transport(const tlt_transport_desc *d) { return check_transport_desc(d, nullptr); }

tlt_status load_transport(tlt_ctx *c, const tlt_transport_desc *d) {
  if (!c || !d) return fail(c ? &c->err : nullptr, TLT_E_ARG, "NULL argument");
  // every host check runs before the device is touched
  tlt_status s = check_transport_desc(d, &c->err);
  if (s != TLT_OK) return s;
  HIPC(c, hipSetDevice(c->device));
  const int N = d->n_vertices;
  int n_pad = 1;
  while (n_pad < N) n_pad <<= 1;
  const int n_cols = d->wavelet == TLT_WAVELET_HAAR ? n_pad : N;
  const int64_t n_rowsW = (int64_t)N * d->K;

  HIPC(c, hipDeviceSynchronize());
  free_all(c);
  c->N = N;
  c->n_pad = n_pad;
  c->n_rows = n_cols;
  c->n_sh = d->n_sh;
  c->n_shp = round_up(d->n_sh, 4);
  c->K = d->K;
  c->nr = d->n_r;
  c->wavelet = d->wavelet;
  c->vdt = d->value_dtype;
  c->tdt = d->transfer_dtype;
  c->n_keep = d->n_keep;
  c->fp64 = d->value_dtype == TLT_F64;
  c->esz = c->fp64 ? 8 : 4;
  c->has_range = d->mat_range != nullptr;
  if (c->has_range) std::memcpy(c->mat_range, d->mat_range, sizeof(c->mat_range));

  const size_t vsz = dtype_size(c->vdt);
  const size_t nnz = (size_t)n_rowsW * (size_t)d->n_keep;
  const TilePlan tp = tile_plan(d, n_cols);
  const int tV = tp.tV;
  const bool want_tiles = tp.want;
  // BF16 tiles carry a second BF16 word for the coarsest columns of every
  // row (their residual), so those products keep ~16 significant bits of
  // W; it needs the float64 values (rows built here, or given as float64)
  const bool head = want_tiles && c->vdt == TLT_BF16 && !c->tune_head_off && (!d->col || d->val_is_f64);
  c->head_cols = head ? std::min(64, n_cols) : 0;
  if ((s = dalloc(c, (void **)&c->col, sizeof(int32_t) * nnz, "transport columns")) != TLT_OK) goto fail_all;
  if ((s = dalloc(c, &c->val, vsz * nnz, "transport values")) != TLT_OK) goto fail_all;
  if ((s = dalloc(c, &c->T, dtype_size(c->tdt) * (size_t)N * c->n_sh + 64, "transfer")) != TLT_OK) goto fail_all;
  if ((s = dalloc(c, &c->area, c->esz * N, "areas")) != TLT_OK) goto fail_all;
  if ((s = dalloc(c, (void **)&c->perm, sizeof(int32_t) * N, "perm")) != TLT_OK) goto fail_all;
  if ((s = dalloc(c, (void **)&c->rn, sizeof(double) * c->nr, "r nodes")) != TLT_OK) goto fail_all;
  if ((s = dalloc(c, (void **)&c->basis, sizeof(double) * c->nr * c->K, "basis")) != TLT_OK) goto fail_all;
  if (head) {
    const size_t rb = sizeof(uint16_t) * (size_t)n_rowsW * c->head_cols;
    if ((s = dalloc(c, (void **)&c->build_res, rb, "BF16 residuals")) != TLT_OK) goto fail_all;
    HIPC(c, hipMemset(c->build_res, 0, rb));
  }
  {
    hipError_t he = hipSuccess;
#define HTRY(x) if ((he = (x)) != hipSuccess) { s = hip_fail(c, he, #x); goto fail_all; }
    HTRY(hipMemcpy(c->perm, d->perm, sizeof(int32_t) * N, hipMemcpyHostToDevice));
    HTRY(hipMemcpy(c->rn, d->r_nodes, sizeof(double) * c->nr, hipMemcpyHostToDevice));
    HTRY(hipMemcpy(c->basis, d->basis, sizeof(double) * c->nr * c->K, hipMemcpyHostToDevice));
    if (c->fp64) {
      HTRY(hipMemcpy(c->area, d->area, sizeof(double) * N, hipMemcpyHostToDevice));
    } else {
      std::vector<float> a(N);
      for (int i = 0; i < N; ++i) a[i] = (float)d->area[i];
      HTRY(hipMemcpy(c->area, a.data(), sizeof(float) * N, hipMemcpyHostToDevice));
    }
    if (d->col) HTRY(hipMemcpy(c->col, d->col, sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
    // float64 host values are rounded to storage on the device, in chunks
    // through a staging buffer (rows given as float64 also write their
    // residual words: the columns are already on the device)
    const size_t stage_elems = (size_t)1 << 24;
    double *stage = nullptr;
    if ((s = dalloc(c, (void **)&stage, sizeof(double) * stage_elems, "staging")) != TLT_OK) goto fail_all;
    auto upload_q = [&](const double *src, void *dst, int dt, size_t n, bool rows) -> hipError_t {
      for (size_t o = 0; o < n; o += stage_elems) {
        const size_t m = std::min(stage_elems, n - o);
        hipError_t e2 = hipMemcpy(stage, src + o, sizeof(double) * m, hipMemcpyHostToDevice);
        if (e2 != hipSuccess) return e2;
        e2 = rows ? launch_quantize_rows(stage, c->col, dst, dt, (int64_t)o, (int64_t)m, d->n_keep,
                                         c->build_res, c->head_cols, 0)
                  : launch_quantize(stage, (char *)dst + o * dtype_size(dt), dt, (int64_t)m, 0);
        if (e2 != hipSuccess) return e2;
        e2 = hipStreamSynchronize(0);
        if (e2 != hipSuccess) return e2;
      }
      return hipSuccess;
    };
    he = upload_q(d->transfer, c->T, c->tdt, (size_t)N * c->n_sh, false);
    if (he == hipSuccess && d->col && d->val_is_f64)
      he = upload_q((const double *)d->val, c->val, c->vdt, nnz, true);
    dfree(stage);
    if (he != hipSuccess) { s = hip_fail(c, he, "uploading transfer / transport values"); goto fail_all; }
    // Rows given in storage precision are uploaded as they are; without
    // rows they are built on the device.  Tiles are then built on the
    // device from the rows.
    if (d->col) {
      if (!d->val_is_f64) HTRY(hipMemcpy(c->val, d->val, vsz * nnz, hipMemcpyHostToDevice));
    } else if ((s = device_build_rows(c, d, n_cols)) != TLT_OK) {
      goto fail_all;
    }
    if (want_tiles && (s = device_build_tiles(c, tV, n_cols)) != TLT_OK) goto fail_all;
    dfree(c->build_res);
    c->build_res = nullptr;
#undef HTRY
  }
  if ((s = ensure_partition(c)) != TLT_OK) goto fail_all;
  if ((s = ensure_P(c, 0)) != TLT_OK) goto fail_all;
  c->loaded = true;
  c->mat_dirty = c->light_dirty = true;
  c->bf16_plain = c->vdt == TLT_BF16 && !(c->tiles && c->head_cols > 0);
  if (c->bf16_plain) {
    c->err = "BF16 storage without the residual words of the coarsest columns";
    return TLT_W_BF16_NO_RESIDUAL;
  }
  return TLT_OK;
fail_all:
  free_all(c);
  return s;
}

tlt_status set_material(tlt_ctx *c, int n_mat, const double *theta_dev, void *stream) {
  (void)stream;   // the values are read (and validated) by render, on its stream
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->loaded) return fail(&c->err, TLT_E_STATE, "set_material before load_transport");
  if (n_mat < 1 || !theta_dev) return fail(&c->err, TLT_E_ARG, "need n_mat >= 1 and a pointer");
  c->theta = theta_dev;
  c->n_mat = n_mat;
  c->mat_dirty = true;
  return TLT_OK;
}

tlt_status tlt_material_status(tlt_ctx *c, void *stream) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  HIPC(c, hipStreamSynchronize((hipStream_t)stream));
  volatile int *f = c->mstat;
  const int bad = f[0], far = f[1], which = f[2];
  f[0] = f[1] = f[2] = 0;
  if (bad)
    return fail(&c->err, TLT_E_ARG,
                "material " + std::to_string(which / 3) + " channel " + std::to_string(which % 3) +
                    ": need sigma_a > 0, sigma_s' > 0, eta >= 1, all finite (its radiance is NaN)");
  if (far) {
    c->err = "material outside the range of the PCA table";
    return TLT_W_MATERIAL_OUT_OF_RANGE;
  }
  return TLT_OK;
}

tlt_status set_lighting(tlt_ctx *c, int n_light, const void *sh_dev) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->loaded) return fail(&c->err, TLT_E_STATE, "set_lighting before load_transport");
  if (n_light < 1 || !sh_dev) return fail(&c->err, TLT_E_ARG, "need n_light >= 1 and a pointer");
  c->sh = sh_dev;
  c->use_E = false;
  c->n_light = n_light;
  c->light_dirty = true;
  c->v_valid = false;
  c->bwd_valid = false;
  return TLT_OK;
}

tlt_status set_irradiance(tlt_ctx *c, int n_light, const void *E_dev) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->loaded) return fail(&c->err, TLT_E_STATE, "set_irradiance before load_transport");
  if (n_light < 1 || !E_dev) return fail(&c->err, TLT_E_ARG, "need n_light >= 1 and a pointer");
  c->E = E_dev;
  c->use_E = true;
  c->n_light = n_light;
  c->light_dirty = true;
  c->v_valid = false;
  c->bwd_valid = false;
  return TLT_OK;
}

tlt_status set_view(tlt_ctx *c, const double *eye, const double *position, const double *normal) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->loaded) return fail(&c->err, TLT_E_STATE, "set_view before load_transport");
  if (!eye) {
    c->view = false;
    return TLT_OK;
  }
  if (!position || !normal) return fail(&c->err, TLT_E_ARG, "need positions and normals");
  HIPC(c, hipSetDevice(c->device));
  std::vector<double> cs(c->N);
  for (int o = 0; o < c->N; ++o) {
    const double d0 = eye[0] - position[3 * (size_t)o], d1 = eye[1] - position[3 * (size_t)o + 1],
                 d2 = eye[2] - position[3 * (size_t)o + 2];
    const double len = std::sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    if (!(len > 0.0) || !std::isfinite(len)) return fail(&c->err, TLT_E_ARG, "eye on a vertex or not finite");
    cs[o] = (normal[3 * (size_t)o] * d0 + normal[3 * (size_t)o + 1] * d1 + normal[3 * (size_t)o + 2] * d2) / len;
  }
  tlt_status s;
  if (!c->view_cos && (s = dalloc(c, &c->view_cos, c->esz * c->N, "view cosines")) != TLT_OK) return s;
  if (c->fp64) {
    HIPC(c, hipMemcpy(c->view_cos, cs.data(), sizeof(double) * c->N, hipMemcpyHostToDevice));
  } else {
    std::vector<float> f(cs.begin(), cs.end());
    HIPC(c, hipMemcpy(c->view_cos, f.data(), sizeof(float) * c->N, hipMemcpyHostToDevice));
  }
  c->view = true;
  return TLT_OK;
}

tlt_status load_spatial(tlt_ctx *c, const tlt_spatial_desc *d) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->loaded) return fail(&c->err, TLT_E_STATE, "load_spatial before load_transport");
  if (!d || !d->col || !d->val) return fail(&c->err, TLT_E_ARG, "need the float64 Step-1 rows");
  HIPC(c, hipSetDevice(c->device));
  if (c->K >= SP_MAX_K) return fail(&c->err, TLT_E_ARG, "spatial compression needs K < 128");
  free_spatial(c);
  SpatialCsr csr;
  const unsigned hw = std::max(1u, std::min(std::thread::hardware_concurrency(), 16u));
  tlt_status s = spatial_build(c->N, c->n_rows, c->K, c->n_keep, d->col, d->val, d->energy,
                               d->levels, d->threads > 0 ? d->threads : (int)hw, csr, &c->err);
  if (s != TLT_OK) return s;
  // work items of at most SEG entries: a longer row is cut into consecutive items
  const int64_t SEG = c->tune_sp_segment ? c->tune_sp_segment : 2048;
  std::vector<int64_t> item_e;
  std::vector<int32_t> u_item((size_t)c->N + 1, 0);
  {
    std::vector<int64_t> ie0, ie1;
    for (int u = 0; u < c->N; ++u) {
      u_item[u] = (int32_t)ie0.size();
      const int64_t a = csr.rowptr[u], b = csr.rowptr[u + 1];
      const int n = b > a ? (int)((b - a + SEG - 1) / SEG) : 1;
      for (int p = 0; p < n; ++p) {
        ie0.push_back(std::min(b, a + p * SEG));
        ie1.push_back(std::min(b, a + (p + 1) * SEG));
      }
    }
    u_item[c->N] = (int32_t)ie0.size();
    item_e = ie0;
    item_e.insert(item_e.end(), ie1.begin(), ie1.end());
  }
  const int n_items = u_item[c->N];
  // w_1^{-1} (Step 5) as a sparse matrix, expanded over the work items of
  // each coefficient's row and stored as padded CSR rows: lanes per output
  // position (tuning, else 32), rows padded to a
  // whole number of entries per lane (a multiple of 4 beyond 8)
  std::vector<int32_t> srp, scol;
  std::vector<double> sw;
  synthesis_build(c->N, csr.sizes, (int)hw, srp, scol, sw);
  int max_len = 1;
  for (int o = 0; o < c->N; ++o) {
    int len = 0;
    for (int e = srp[o]; e < srp[o + 1]; ++e) len += u_item[scol[e] + 1] - u_item[scol[e]];
    max_len = std::max(max_len, len);
  }
  const int syn_lanes = c->tune_sp_syn_lanes ? c->tune_sp_syn_lanes : 32;
  const int per = (max_len + syn_lanes - 1) / syn_lanes;        // entries per lane
  const int syn_len = (per <= 8 ? per : (per + 3) / 4 * 4) * syn_lanes;
  std::vector<int32_t> pad_col((size_t)syn_len * c->N, 0);
  std::vector<double> pad_w((size_t)syn_len * c->N, 0.0);
  for (int o = 0; o < c->N; ++o) {
    size_t d = (size_t)o * syn_len;
    for (int e = srp[o]; e < srp[o + 1]; ++e)
      for (int it = u_item[scol[e]]; it < u_item[scol[e] + 1]; ++it) {
        pad_col[d] = it;
        pad_w[d++] = sw[e];
      }
  }
  const int64_t nnz = csr.rowptr[c->N];
  const size_t n1 = std::max<int64_t>(nnz, 1);
  if ((s = dalloc(c, (void **)&c->sp_col, sizeof(uint32_t) * n1, "spatial columns")) != TLT_OK ||
      (s = dalloc(c, &c->sp_val, c->esz * n1, "spatial values")) != TLT_OK ||
      (s = dalloc(c, (void **)&c->sp_item_e, sizeof(int64_t) * item_e.size(), "spatial items")) != TLT_OK ||
      (s = dalloc(c, (void **)&c->sp_syn_col, sizeof(int32_t) * pad_col.size(), "synthesis")) != TLT_OK ||
      (s = dalloc(c, &c->sp_syn_w, c->esz * pad_w.size(), "synthesis")) != TLT_OK) {
    free_spatial(c);
    return s;
  }
  hipError_t e = hipSuccess;
  if (nnz > 0) e = hipMemcpy(c->sp_col, csr.col.data(), sizeof(uint32_t) * nnz, hipMemcpyHostToDevice);
  auto put = [&](void *dst, const std::vector<double> &v) {
    if (c->fp64) return hipMemcpy(dst, v.data(), sizeof(double) * v.size(), hipMemcpyHostToDevice);
    std::vector<float> f(v.begin(), v.end());
    return hipMemcpy(dst, f.data(), sizeof(float) * f.size(), hipMemcpyHostToDevice);
  };
  if (e == hipSuccess && nnz > 0) e = put(c->sp_val, csr.val);
  if (e == hipSuccess)
    e = hipMemcpy(c->sp_item_e, item_e.data(), sizeof(int64_t) * item_e.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(c->sp_syn_col, pad_col.data(), sizeof(int32_t) * pad_col.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = put(c->sp_syn_w, pad_w);
  if (e != hipSuccess) {
    free_spatial(c);
    return hip_fail(c, e, "load_spatial upload");
  }
  c->sp_items = n_items;
  c->sp_syn_len = syn_len;
  c->sp_syn_lanes = syn_lanes;
  c->sp_mean_item = n_items > 0 ? (double)nnz / n_items : 0.0;
  c->sp_nnz = nnz;
  c->sp_levels = (int)csr.sizes.size();
  for (int i = 0; i < c->sp_levels; ++i) c->sp_sizes[i] = csr.sizes[i];
  c->sp_rowptr = std::move(csr.rowptr);
  c->sp_nnz_k = std::move(csr.nnz_k);
  c->sp_energy = std::move(csr.energy_kept);
  c->spatial = true;
  return TLT_OK;
}

tlt_status tlt_spatial_info(tlt_ctx *c, int64_t *nnz, int32_t *levels, int64_t *nnz_k,
                            double *energy_kept) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->spatial) return fail(&c->err, TLT_E_STATE, "no spatial compression loaded");
  if (nnz) *nnz = c->sp_nnz;
  if (levels) *levels = c->sp_levels;
  for (int k = 0; k < c->K; ++k) {
    if (nnz_k) nnz_k[k] = c->sp_nnz_k[k];
    if (energy_kept) energy_kept[k] = c->sp_energy[k];
  }
  return TLT_OK;
}

tlt_status tlt_read_spatial(tlt_ctx *c, int64_t u0, int64_t n_u, int64_t *rowptr_out,
                            uint32_t *col_out, double *val_out, int64_t capacity) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->spatial) return fail(&c->err, TLT_E_STATE, "no spatial compression loaded");
  if (u0 < 0 || n_u < 0 || u0 + n_u > c->N || !rowptr_out)
    return fail(&c->err, TLT_E_ARG, "rows out of range");
  const int64_t base = c->sp_rowptr[u0];
  for (int64_t i = 0; i <= n_u; ++i) rowptr_out[i] = c->sp_rowptr[u0 + i] - base;
  const int64_t m = rowptr_out[n_u];
  if (m > capacity) return fail(&c->err, TLT_E_ARG, "capacity below the entries of these rows");
  if (m == 0) return TLT_OK;
  if (!col_out || !val_out) return fail(&c->err, TLT_E_ARG, "NULL output");
  HIPC(c, hipDeviceSynchronize());
  HIPC(c, hipMemcpy(col_out, c->sp_col + base, sizeof(uint32_t) * m, hipMemcpyDeviceToHost));
  if (c->fp64) {
    HIPC(c, hipMemcpy(val_out, (const double *)c->sp_val + base, sizeof(double) * m, hipMemcpyDeviceToHost));
  } else {
    std::vector<float> f(m);
    HIPC(c, hipMemcpy(f.data(), (const float *)c->sp_val + base, sizeof(float) * m, hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < m; ++i) val_out[i] = f[i];
  }
  return TLT_OK;
}

tlt_status render(tlt_ctx *c, void *B, void *stream, int flags) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->loaded) return fail(&c->err, TLT_E_STATE, "render before load_transport");
  if (!(c->use_E ? c->E : c->sh) || !c->theta)
    return fail(&c->err, TLT_E_STATE, "render before set_lighting (or set_irradiance) / set_material");
  if (!B) return fail(&c->err, TLT_E_ARG, "B is NULL");
  if (c->n_light != c->n_mat && c->n_light != 1 && c->n_mat != 1)
    return fail(&c->err, TLT_E_ARG, "n_light and n_mat must match or one must be 1");
  if (flags & ~(TLT_SAVE_FOR_BACKWARD | TLT_FORCE_FULL | TLT_PLAIN_ROWS | TLT_FOLDED_LIGHTING |
                TLT_SPATIAL | TLT_KEEP_TERMS))
    return fail(&c->err, TLT_E_ARG, "unknown flags");
  const bool spatial = flags & TLT_SPATIAL;
  if (spatial && (flags & (TLT_SAVE_FOR_BACKWARD | TLT_KEEP_TERMS | TLT_PLAIN_ROWS | TLT_FOLDED_LIGHTING)))
    return fail(&c->err, TLT_E_ARG,
                "TLT_SPATIAL excludes TLT_SAVE_FOR_BACKWARD, TLT_KEEP_TERMS, TLT_PLAIN_ROWS and "
                "TLT_FOLDED_LIGHTING");
  if (spatial && !c->spatial) return fail(&c->err, TLT_E_STATE, "TLT_SPATIAL before load_spatial");
  if ((flags & TLT_FOLDED_LIGHTING) && (flags & (TLT_KEEP_TERMS | TLT_PLAIN_ROWS)))
    return fail(&c->err, TLT_E_ARG, "TLT_FOLDED_LIGHTING excludes TLT_KEEP_TERMS and TLT_PLAIN_ROWS");
  if ((flags & TLT_FOLDED_LIGHTING) && c->use_E)
    return fail(&c->err, TLT_E_ARG, "TLT_FOLDED_LIGHTING needs SH lighting, not a supplied irradiance");
  hipStream_t st = (hipStream_t)stream;
  tlt_status s;
  if ((s = ensure_columns(c)) != TLT_OK) return s;
  const bool save = flags & TLT_SAVE_FOR_BACKWARD;
  const bool keep = flags & TLT_KEEP_TERMS;
  const bool full = flags & TLT_FORCE_FULL;
  const bool use_tiles = c->tiles && !(flags & TLT_PLAIN_ROWS);
  if (keep && (s = ensure_V(c)) != TLT_OK) return s;
  // the adjoint differentiates this render: it reads P, the weights and
  // the lighting buffer of this render (no extra writes here)
  c->bwd_valid = false;
  Cols cols{c->C, c->n_out, c->n_light, c->n_mat};
  bool bf16_without_residual = false;
  const bool do_gk = c->mat_dirty || full;
  const bool relight = c->light_dirty || full || !(c->v_valid);
  PrepArgs a = prep_args(c, c->Cs, cols);
  if (do_gk) {
    a.n_gk_blocks = c->n_mat * 3;
    a.theta = c->theta;
    a.g64 = c->g64;
    a.dg64 = c->dg64;
    a.gcol = c->gcol;
  }
  if (flags & TLT_FOLDED_LIGHTING) {
    // g_k when the material changed, then the folded product
    if (!c->have_P && (s = ensure_P(c, st)) != TLT_OK) return s;
    if (!c->tune_fold_fp32 && (s = ensure_P16(c, st)) != TLT_OK) return s;
    if (do_gk) {
      StageTimer t(c, 0, st);
      HIPC(c, launch_prep(a, st));
    }
    const size_t need = folded_scratch_bytes(c->K, c->Psh, c->Cs, c->fp64);
    if (c->fold_bytes < need) {
      dfree(c->fold);
      c->fold_bytes = 0;
      if ((s = dalloc(c, &c->fold, need, "folded lighting weights")) != TLT_OK) return s;
      c->fold_bytes = need;
    }
    StageTimer t(c, 2, st);
    const bool p16 = c->P16 && !c->tune_fold_fp32;
    HIPC(c, launch_folded(c->P, c->Psh, c->n_sh, c->K, c->gcol, c->Cs, c->sh, cols, c->N, B, c->fp64,
                          c->fold, st, p16 ? c->P16 : nullptr, c->p16_inv));
    c->v_valid = false;
  } else if (!relight && c->V && !spatial) {
    // material-only edit: reuse the per-term transport v_k kept by the last
    // full render (TLT_KEEP_TERMS)
    if (do_gk) {
      StageTimer t(c, 0, st);
      HIPC(c, launch_prep(a, st));
    }
    StageTimer t(c, 4, st);
    HIPC(c, launch_combine(c->V, c->Cs, c->gcol, c->K, c->N, c->C, B, c->fp64, st));
  } else {
    a.n_tl_blocks = c->n_chunks * (c->Cs / 16);
    if (c->use_E) {
      a.E = c->E;
      a.perm = c->perm;
    } else {
      a.sh = c->sh;
      if (c->wavelet == TLT_WAVELET_HAAR && !c->tune_irr_haar && c->Cs <= 32) {
        // Ehat = G L: one matrix product per chunk, no Haar levels.  Each
        // 16-column tile of a chunk reads the chunk's G rows (padded length,
        // float32), so this pays only for narrow launches; wide ones keep
        // the per-frame Haar of the compact transfer rows.
        if ((s = ensure_G(c, st)) != TLT_OK) return s;
        a.T = c->Gmat;
        a.tdt = c->fp64 ? TLT_F64 : TLT_F32;
        a.t_ld = c->G_ld;
        a.t_rows = c->n_rows;
        a.area = nullptr;
        a.haar = 0;
      }
    }
    a.ehat = c->ehat;
    a.partial = c->partial;
    a.ehat2 = c->ehat2;
    a.split = c->vdt == TLT_BF16 ? 1 : 2;
    const bool rows_kernel = !use_tiles && !spatial;
    bf16_without_residual = c->vdt == TLT_BF16 && !spatial && (rows_kernel || c->bf16_plain);
    if (rows_kernel && (s = ensure_partition(c)) != TLT_OK) return s;
    if (c->n_zero > 0 && rows_kernel) {
      a.B = B;
      a.zero_v = c->zero_v;
      a.n_zero = c->n_zero;
      a.n_zero_blocks = std::max(1, std::min(64, (c->n_zero * c->C + 255) / 256));
    }
    {
      StageTimer t(c, 1, st);
      HIPC(c, launch_prep(a, st));
    }
    SpatialArgs spa;
    std::memset(&spa, 0, sizeof(spa));
    {
      StageTimer t(c, 2, st);
      if (spatial) {
        const size_t pb = c->esz * (size_t)std::max(c->sp_items, 1) * c->C;
        if (c->sp_part_bytes < pb) {
          dfree(c->sp_part);
          c->sp_part_bytes = 0;
          if ((s = dalloc(c, &c->sp_part, pb, "spatial partial sums")) != TLT_OK) return s;
          c->sp_part_bytes = pb;
        }
        spa.col = c->sp_col;
        spa.val = c->sp_val;
        spa.n_items = c->sp_items;
        // built-in shape (measured at haar-f32-10242): a wave per item of at
        // most 2048 entries, eight entries per lane and pass
        spa.lanes_per_item = c->tune_sp_lanes ? c->tune_sp_lanes : 64;
        spa.unroll = c->tune_sp_unroll ? c->tune_sp_unroll : 8;
        spa.item_e0 = c->sp_item_e;
        spa.item_e1 = c->sp_item_e + c->sp_items;
        spa.part = c->sp_part;
        spa.syn_len = c->sp_syn_len;
        spa.syn_lanes = c->sp_syn_lanes;
        spa.syn_col = c->sp_syn_col;
        spa.syn_w = c->sp_syn_w;
        spa.ehat = c->ehat;
        spa.gcol = c->gcol;
        spa.Cs = c->Cs;
        spa.C = c->C;
        spa.K = c->K;
        spa.N = c->N;
        spa.perm = c->perm;
        spa.B = B;
        HIPC(c, launch_spatial_rows(spa, c->fp64, st));
      } else if (use_tiles) {
        HIPC(c, launch_tiles(tile_args(c, c->ehat, c->ehat2, c->Cs, c->C, c->gcol, B,
                                       keep ? c->V : nullptr, c->Cs),
                             c->vdt, st));
      } else {
        if ((s = ensure_partition(c)) != TLT_OK) return s;
        StreamArgs sa = stream_args(c, c->ehat, c->Cs, c->C, c->gcol, B, keep ? c->V : nullptr, c->Cs);
        HIPC(c, launch_stream(sa, c->vdt, c->fp64, c->cpl, st));
      }
    }
    if (spatial) {
      StageTimer t(c, 5, st);
      HIPC(c, launch_spatial_synthesis(spa, c->fp64, st));
    }
    c->v_valid = keep && !spatial;
  }
  c->bwd_valid = save && !spatial && !c->use_E;
  if (c->view) HIPC(c, launch_view(B, c->view_cos, c->theta, cols, c->N, c->perm, c->fp64, st));
  c->mat_dirty = false;
  c->light_dirty = false;
  if (bf16_without_residual) {
    c->err = "BF16 transport product without the residual words of the coarsest columns";
    return TLT_W_BF16_NO_RESIDUAL;
  }
  return TLT_OK;
}

// Checks of the adjoint entry points.
static tlt_status backward_check(tlt_ctx *c, const void *dB, const void *dSH, const double *dTheta) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->loaded || !c->bwd_valid || !c->have_P || c->mat_dirty || c->light_dirty)
    return fail(&c->err, TLT_E_STATE,
                "render_backward needs a render with TLT_SAVE_FOR_BACKWARD of the current inputs");
  if (c->use_E)
    return fail(&c->err, TLT_E_STATE, "render_backward needs SH lighting, not a supplied irradiance");
  if (c->view)
    return fail(&c->err, TLT_E_STATE, "render_backward is for the radiance without the view factor");
  if (!dB || !dSH || !dTheta) return fail(&c->err, TLT_E_ARG, "NULL gradient pointer");
  return TLT_OK;
}

static tlt_status backward_launch(tlt_ctx *c, const void *dB, void *dSH, double *dTheta,
                                  void *scratch_ptr, size_t scratch_bytes, hipStream_t st) {
  Cols cols{c->C, c->n_out, c->n_light, c->n_mat};
  HIPC(c, launch_adjoint(dB, c->P, c->Psh, c->gcol, c->Cs, c->sh, c->dg64, c->N, c->K, c->n_sh, cols,
                         c->fp64, scratch_ptr, scratch_bytes, dSH, dTheta, st));
  return TLT_OK;
}

tlt_status render_backward(tlt_ctx *c, const void *dB, void *dSH, double *dTheta, void *stream) {
  tlt_status s = backward_check(c, dB, dSH, dTheta);
  if (s != TLT_OK) return s;
  const size_t need = adjoint_partial_bytes(c->N, c->K, c->n_sh, c->C, c->fp64);
  if (c->adj_bytes < need) {
    dfree(c->adj);
    c->adj_bytes = 0;
    if ((s = dalloc(c, &c->adj, need, "adjoint partials")) != TLT_OK) return s;
    c->adj_bytes = need;
  }
  StageTimer t(c, 3, (hipStream_t)stream);
  return backward_launch(c, dB, dSH, dTheta, c->adj, c->adj_bytes, (hipStream_t)stream);
}

tlt_status render_backward_noalloc(tlt_ctx *c, const void *dB, void *dSH, double *dTheta,
                                   void *stream) {
  tlt_status s = backward_check(c, dB, dSH, dTheta);
  if (s != TLT_OK) return s;
  const size_t need = adjoint_partial_bytes(c->N, c->K, c->n_sh, c->C, c->fp64);
  if (need > TLT_NOALLOC_SCRATCH_BYTES)
    return fail(&c->err, TLT_E_ARG,
                "the adjoint of this launch needs " + std::to_string(need) +
                    " bytes of partial sums, more than the static buffer of render_backward_noalloc (" +
                    std::to_string((size_t)TLT_NOALLOC_SCRATCH_BYTES) + " bytes); use render_backward");
  if (!c->scratch_dev) return fail(&c->err, TLT_E_STATE, "no static scratch address for this device");
  // no stage timer: it may create events
  return backward_launch(c, dB, dSH, dTheta, c->scratch_dev, TLT_NOALLOC_SCRATCH_BYTES,
                         (hipStream_t)stream);
}

tlt_status tlt_set_tuning(tlt_ctx *c, int32_t key, int32_t value) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (value < 0) return fail(&c->err, TLT_E_ARG, "tuning values are >= 0 (0 = built-in choice)");
  switch (key) {
    case TLT_TUNE_TILE_CHUNK: c->tune_tile_chunk = value; break;
    case TLT_TUNE_BF16_HEAD:
      if (value > 1) return fail(&c->err, TLT_E_ARG, "BF16 head flag must be 0 or 1");
      c->tune_head_off = value;
      break;
    case TLT_TUNE_TILE_SPARSE:
      if (value > 2) return fail(&c->err, TLT_E_ARG, "tile form must be 0, 1 or 2");
      c->tune_tile_sparse = value;
      break;
    case TLT_TUNE_FOLDED_FP32:
      if (value > 1) return fail(&c->err, TLT_E_ARG, "folded precision flag must be 0 or 1");
      c->tune_fold_fp32 = value;
      break;
    case TLT_TUNE_IRRADIANCE_HAAR:
      if (value > 1) return fail(&c->err, TLT_E_ARG, "irradiance flag must be 0 or 1");
      c->tune_irr_haar = value;
      break;
    case TLT_TUNE_TILE_SHAPE:
      if (value != 0 && value != 231 && value != 241 && value != 432 && value != 442)
        return fail(&c->err, TLT_E_ARG, "tile shape must be 231, 241, 432 or 442");
      c->tune_tile_shape = value;
      break;
    case TLT_TUNE_STREAM_WAVES_PER_CU: c->tune_waves_per_cu = value; break;
    case TLT_TUNE_STREAM_EPL:
      if (value != 0 && value != 4 && value != 8 && value != 16)
        return fail(&c->err, TLT_E_ARG, "entries per lane must be 4, 8 or 16");
      c->tune_stream_epl = value;
      break;
    case TLT_TUNE_STREAM_NT:
      if (value > 1) return fail(&c->err, TLT_E_ARG, "non-temporal flag must be 0 or 1");
      c->tune_stream_nt = value;
      break;
    case TLT_TUNE_SPATIAL_LANES:
      if (value != 0 && value != 16 && value != 32 && value != 64)
        return fail(&c->err, TLT_E_ARG, "lanes per item must be 16, 32 or 64");
      c->tune_sp_lanes = value;
      break;
    case TLT_TUNE_SPATIAL_UNROLL:
      if (value != 0 && value != 4 && value != 8 && value != 16)
        return fail(&c->err, TLT_E_ARG, "entries per lane must be 4, 8 or 16");
      c->tune_sp_unroll = value;
      break;
    case TLT_TUNE_SPATIAL_SYNTH_LANES:
      if (value != 0 && value != 8 && value != 16 && value != 32)
        return fail(&c->err, TLT_E_ARG, "lanes per output position must be 8, 16 or 32");
      c->tune_sp_syn_lanes = value;
      break;
    case TLT_TUNE_SPATIAL_SEGMENT:
      if (value != 0 && (value < 64 || value > (1 << 20)))
        return fail(&c->err, TLT_E_ARG, "segment length must be in 64 .. 2^20");
      c->tune_sp_segment = value;
      break;
    default: return fail(&c->err, TLT_E_ARG, "unknown tuning key");
  }
  return TLT_OK;
}

tlt_status tlt_read_probe(const void *buf, int64_t bytes, uint32_t *out, int blocks, void *stream) {
  if ((!buf && bytes > 0) || !out || bytes < 0 || bytes % 16 || blocks < 1)
    return fail(nullptr, TLT_E_ARG, "bad arguments");
  const hipError_t e = launch_read_probe(buf, bytes, out, blocks, (hipStream_t)stream);
  if (e != hipSuccess) return fail(nullptr, TLT_E_HIP, std::string("read probe: ") + hipGetErrorString(e));
  return TLT_OK;
}

tlt_status tlt_profile_enable(tlt_ctx *c, int mode) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (mode < 0 || mode > 2) return fail(&c->err, TLT_E_ARG, "mode must be 0, 1 or 2");
  if (mode == 1) {
    prof_drain(c);
    for (int i = 0; i < 6; ++i) {
      c->prof_ms[i] = 0.0;
      c->prof_n[i] = 0;
    }
  }
  c->prof = mode != 0;
  return TLT_OK;
}

tlt_status tlt_profile_read(tlt_ctx *c, int stage, double *total_ms, int64_t *launches) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (stage < 0 || stage > 5) return fail(&c->err, TLT_E_ARG, "stage must be in 0..5");
  prof_drain(c);
  if (total_ms) *total_ms = c->prof_ms[stage];
  if (launches) *launches = c->prof_n[stage];
  return TLT_OK;
}

tlt_status tlt_read_rows(tlt_ctx *c, int64_t n_rows, const int64_t *rows, int32_t *col_out,
                         double *val_out) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->loaded) return fail(&c->err, TLT_E_STATE, "no transport loaded");
  if (n_rows < 0 || (n_rows > 0 && (!rows || !col_out || !val_out)))
    return fail(&c->err, TLT_E_ARG, "bad arguments");
  const int64_t total = (int64_t)c->N * c->K;
  const size_t vsz = dtype_size(c->vdt);
  std::vector<unsigned char> raw(vsz * c->n_keep);
  HIPC(c, hipDeviceSynchronize());
  for (int64_t i = 0; i < n_rows; ++i) {
    if (rows[i] < 0 || rows[i] >= total) return fail(&c->err, TLT_E_ARG, "row out of range");
    const size_t off = (size_t)rows[i] * c->n_keep;
    HIPC(c, hipMemcpy(col_out + i * c->n_keep, c->col + off, sizeof(int32_t) * c->n_keep,
                      hipMemcpyDeviceToHost));
    HIPC(c, hipMemcpy(raw.data(), (char *)c->val + off * vsz, vsz * c->n_keep, hipMemcpyDeviceToHost));
    for (int64_t e = 0; e < c->n_keep; ++e) val_out[i * c->n_keep + e] = widen(raw.data(), c->vdt, e);
  }
  return TLT_OK;
}

tlt_status tlt_tile_info(tlt_ctx *c, int32_t *vertices, int64_t *blocks, int64_t *entries,
                         int64_t *fragments, int64_t *value_bytes, int32_t *sparse) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->loaded || !c->tiles) return fail(&c->err, TLT_E_STATE, "no tiles loaded");
  if (vertices) *vertices = c->tV;
  if (blocks) *blocks = c->t_blocks;
  if (entries) {
    int64_t n = 0;
    HIPC(c, hipMemcpy(&n, c->t_off + c->t_blocks, sizeof(int64_t), hipMemcpyDeviceToHost));
    *entries = n;
  }
  if (fragments) *fragments = c->t_frags;
  if (value_bytes) *value_bytes = (int64_t)c->t_val_bytes;
  if (sparse) *sparse = c->t_sparse ? 1 : 0;
  return TLT_OK;
}

tlt_status tlt_read_state(tlt_ctx *c, int which, void *out, size_t *bytes, int *c_stride) {
  if (!c) return fail(nullptr, TLT_E_ARG, "ctx is NULL");
  if (!c->ehat) return fail(&c->err, TLT_E_STATE, "nothing rendered yet");
  const void *src = nullptr;
  size_t n = 0;
  switch (which) {
    case 0: src = c->ehat; n = c->esz * (size_t)c->n_rows * c->Cs; break;
    case 1: src = c->g64; n = sizeof(double) * c->n_mat * 3 * c->K; break;
    case 2: src = c->dg64; n = sizeof(double) * c->n_mat * 9 * c->K; break;
    default: return fail(&c->err, TLT_E_ARG, "unknown state id");
  }
  if (c_stride) *c_stride = c->Cs;
  if (bytes) *bytes = n;
  if (!out) return TLT_OK;
  HIPC(c, hipDeviceSynchronize());
  HIPC(c, hipMemcpy(out, src, n, hipMemcpyDeviceToHost));
  return TLT_OK;
}

}  // extern "C"
