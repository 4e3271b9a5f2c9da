/*
 * tlt.h -- C ABI of the MI355X translucent-transport library (libtlt.so).
 *
 * Per-frame radiance of a translucent object under the dipole diffusion
 * model with a PCA-factorised material function and Haar-compressed
 * precomputed transport (Wang, Hua, Huo, Bao, "Real-time Rendering and
 * Editing of Scattering Effects for Translucent Objects"):
 *
 *   E[q,i,ch]    = sum_lm T[i,lm] L[light(q),lm,ch]                 (Eq. 6)
 *   Ehat[q,:,ch] = Haar(pad(A o E[q,:,ch]))  over Morton order      (Eq. 8)
 *   g[m,ch,k]    = sum_n R_d(r_n; theta[m,ch]) b_k[n]     (Sec. 2.2, Eq. 4)
 *   B[q,v,ch]    = sum_k g[mat(q),ch,k] sum_{j in S(o,k)} W_k[o,j] Ehat[q,j,ch]
 *                  with v = perm[o]                (Eq. 7, 8; Sec. 4 Steps 1-4)
 *
 * Column convention: a launch renders n_out = max(n_light, n_mat) sets of
 * three RGB channels; set q uses lighting light(q) = (n_light > 1 ? q : 0)
 * and material mat(q) = (n_mat > 1 ? q : 0).  n_light and n_mat must be
 * equal or one of them must be 1.
 *
 * Precision: a transport stored in F64 runs entirely in float64 (E, Ehat,
 * accumulation, B, gradients).  Any other storage (F32, BF16, F16) runs in
 * float32 with float32 accumulation; the material weights g are always
 * evaluated in float64 on the GPU.
 *
 * Errors: every call returns a tlt_status; nothing aborts or throws across
 * the ABI.  tlt_last_error() gives a message for the last failing call on a
 * context (or, for ctx == NULL, on the calling thread).  GPU work is
 * asynchronous on the caller's HIP stream: launch failures return
 * TLT_E_HIP, faults inside kernels surface at a later synchronising call.
 * A context is not thread-safe; use one per thread.
 */
#ifndef TLT_H
#define TLT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tlt_ctx tlt_ctx;

typedef enum {
  TLT_OK = 0,
  TLT_W_MATERIAL_OUT_OF_RANGE = 1, /* warning: material outside the PCA table */
  TLT_W_BF16_NO_RESIDUAL = 2,      /* warning: BF16 products without the residual words */
  TLT_E_ARG = -1,                  /* bad argument, shape or value */
  TLT_E_STATE = -2,                /* call out of order */
  TLT_E_OOM = -3,                  /* device or host allocation failed */
  TLT_E_HIP = -4,                  /* HIP runtime error */
  TLT_E_FORMAT = -5                /* malformed transport (indices, sizes) */
} tlt_status;

enum { TLT_F64 = 0, TLT_F32 = 1, TLT_BF16 = 2, TLT_F16 = 3 };
enum { TLT_WAVELET_NONE = 0, TLT_WAVELET_HAAR = 1 };
enum {
  TLT_SAVE_FOR_BACKWARD = 1, /* render_backward may differentiate this render (no extra work) */
  TLT_FORCE_FULL = 2,        /* recompute every stage, ignoring dirty flags */
  TLT_PLAIN_ROWS = 4,        /* use the (column, value) row kernel even when tiles exist */
  TLT_FOLDED_LIGHTING = 8,   /* relight through P_k = W_k H (A o T): B = sum_k g_k P_k L */
  TLT_SPATIAL = 16,          /* render through the spatially compressed transport (load_spatial) */
  TLT_KEEP_TERMS = 32        /* keep v_k[v,c] so a material-only edit reruns Steps 3-4 only */
};
enum { TLT_LAYOUT_AUTO = 0, TLT_LAYOUT_ROWS = 1, TLT_LAYOUT_TILES = 2 };

/*
 * Host-side geometry precompute (no GPU work).
 *
 * From a closed triangle mesh computes, all in float64:
 *   - Morton order: perm[p] = vertex id at position p of the 1-D wavelet
 *     domain; coordinates quantised to 21 bits over the bounding box,
 *     bits interleaved x,y,z (x most significant), stable on equal keys
 *     (replaces the flattened quadtrees of Sec. 3.1);
 *   - per-vertex area A_i = 1/3 of the incident triangle areas (dA, Eq. 6);
 *   - vertex normals (area-weighted face normals, normalised);
 *   - SH transfer T[i,lm] = Ahat_l Y_lm(n_i) of the unshadowed clamped
 *     cosine (E of Eq. 6 with visibility 1), real orthonormal SH without
 *     the Condon-Shortley phase, index l*l+l+m;
 *   - r nodes r_n = r_max (n/(n_r-1))^2 and the PCA basis b_k: the first K
 *     right singular vectors of M[material][node] = R_d(r_node; material)
 *     over the material grid (Eq. 5, Sec. 2.2), each signed so that its
 *     entry of largest magnitude is positive.  Grid: sigma_a and sigma_s'
 *     log-spaced over [lo,hi], eta linear, with n points each.
 * All output arrays are caller-allocated host memory; arrays in Morton
 * order are indexed by position p.  Errors: TLT_E_ARG for bad sizes or
 * degenerate meshes (zero-area vertex, zero normal).
 */
typedef struct {
  int32_t n_vertices;        /* N >= 2 */
  int32_t n_faces;
  const double *vertices;    /* [N][3], mm */
  const int32_t *faces;      /* [n_faces][3], counter-clockwise from outside */
  int32_t n_sh;              /* (lmax+1)^2 with lmax in 0..7 */
  int32_t K;                 /* basis functions kept, 1..n_r */
  int32_t n_r;               /* r nodes, 2..1024 (256 by default) */
  double r_max;              /* >= every vertex-to-vertex distance, mm */
  double mat_lo[3];          /* sigma_a, sigma_s' (1/mm), eta */
  double mat_hi[3];
  int32_t mat_n[3];          /* grid points per parameter, each >= 1 */
  /* outputs */
  int32_t *perm;             /* [N] */
  double *position;          /* [N][3]   Morton order */
  double *area;              /* [N]      Morton order */
  double *normal;            /* [N][3]   Morton order */
  double *transfer;          /* [N][n_sh] Morton order */
  double *r_nodes;           /* [n_r] */
  double *basis;             /* [K][n_r] */
  double *singular_values;   /* [min(n_mat, n_r)] or NULL */
} tlt_scene;

tlt_status tlt_prepare_scene(tlt_scene *scene);

/*
 * Host-only: the float64 transport rows for selected output points -- the
 * same rows, operation for operation, that load_transport builds on the
 * device when desc->col == NULL (usable to precompute rows offline).  For each of the n_rows
 * Morton positions rows[i] and each k < K, writes the n_keep kept (column,
 * value) pairs of row (rows[i], k) to col_out/val_out [n_rows][K][n_keep],
 * columns ascending (precompute Step 1 of Sec. 3.2; Eq. 7 and 8).
 * position [N][3] Morton order; n_cols = n_pad (HAAR) or N (NONE).
 * TLT_E_ARG for bad sizes or rows out of range.
 */
tlt_status tlt_build_rows(int32_t n_vertices, int32_t n_cols, int32_t K, int32_t n_r,
                          int32_t wavelet, int64_t n_keep, const double *position,
                          const double *r_nodes, const double *basis, int64_t n_rows,
                          const int64_t *rows, int32_t *col_out, double *val_out);

/*
 * Transport description for load_transport.  Host pointers, caller-owned,
 * read only during the call.
 *
 * Rows are ordered (o, k) with o the Morton position: row = o*K + k.  Each
 * row holds n_keep (column, value) pairs with strictly ascending columns.
 * With wavelet HAAR column j indexes the orthonormal Haar coefficient of
 * the zero-padded Morton list (layout [s0, d0, d1[0..1], ...]; Eq. 8) and
 * the row keeps the n_keep coefficients of largest magnitude (Sec. 3.2,
 * precompute Step 1; ties to the lower j).  With wavelet NONE column j is
 * the Morton position itself (the plain matrix of Eq. 7).  Row values are
 * btilde_k(|x_o - x_j|): the basis b_k interpolated linearly between the
 * r nodes, i.e. the area weight is applied to the irradiance side.
 *
 * col == NULL: the rows are computed on the device in float64 from
 *   `position`, `r_nodes` and `basis`, then stored in value_dtype (rounded
 *   to nearest even, 16-bit types via float32).  With BF16 storage and
 *   tiles, each row's entries in the 64 coarsest Haar columns (levels 0-5,
 *   j < 64; those that dominate the rounding error of the product) also
 *   keep the BF16 rounding of their residual W - bf16(W), stored in the
 *   tiles as extra entries of the same columns, so that in the tile
 *   product these entries carry ~16 significant bits; the plain rows hold
 *   the BF16 values alone.  TLT_TUNE_BF16_HEAD = 1 turns this off.  Supported for n_cols <=
 *   2^20 with n_keep == n_cols or n_keep <= 8192, else TLT_E_ARG; a failed
 *   internal consistency check of the selection gives TLT_E_STATE.
 * col != NULL: col/val are taken as given; every column is checked to lie
 *   in [0, n_cols) and rows to ascend, else TLT_E_FORMAT.  val holds
 *   value_dtype values (val_is_f64 = 0), or float64 values (val_is_f64 =
 *   1) that the library rounds to value_dtype on the device as the device
 *   build does -- with BF16 tiles they then also keep the residual words of
 *   the coarsest columns (the rows tlt_build_rows writes, loaded this way,
 *   give the same transport as col == NULL).
 * Warning TLT_W_BF16_NO_RESIDUAL (the transport is loaded and usable): BF16
 *   storage whose tiles carry no residual words (rows given as BF16 values,
 *   layout ROWS, tiles impossible, or TLT_TUNE_BF16_HEAD = 1).  Plain BF16
 *   values keep 8 significant bits of every coefficient; at 2% kept on
 *   40962 vertices the worst output set then reaches ~5e-3 relative error
 *   against the float64 operator, at the edge of the 5e-3 bound, against
 *   ~2e-3 with the residual words.
 * n_cols = n_pad (HAAR, n_pad = next power of two >= N) or N (NONE).
 *
 * Layout.  The rows are always kept as (column, value) pairs (the plain
 * form).  Unless layout is ROWS or the storage is F64, the library also
 * re-encodes them as block-dense tiles: V Morton-consecutive vertices
 * (V*K rows: 48..128 and a multiple of 16, or 256 with 16-bit storage;
 * tile_vertices, or by default 48..64 rows for F32 storage and up to 128
 * for 16-bit storage) share the
 * sorted union of their kept columns and are stored densely over it
 * (zeros where a row did not keep a column), in the
 * operand order of the 16x16 matrix instructions.  Both layouts hold the
 * same kept coefficients; render uses the tiles unless TLT_PLAIN_ROWS.
 * The library keeps its own device copies until tlt_destroy or the next
 * load_transport.  Material and lighting state are reset.
 */
typedef struct {
  int32_t n_vertices;
  int32_t n_pad;
  int32_t n_sh;
  int32_t K;
  int32_t n_r;
  int32_t wavelet;           /* TLT_WAVELET_* */
  int32_t value_dtype;       /* storage of W: TLT_F64/F32/BF16/F16 */
  int32_t transfer_dtype;    /* storage of T: same set; F64 iff value_dtype F64 */
  int64_t n_keep;            /* entries per row, 1..n_cols */
  const int32_t *col;        /* [N*K][n_keep] or NULL */
  const void *val;           /* [N*K][n_keep] in value_dtype, or NULL */
  const double *position;    /* [N][3] Morton order (needed when col == NULL) */
  const double *transfer;    /* [N][n_sh] Morton order */
  const double *area;        /* [N] Morton order */
  const int32_t *perm;       /* [N] */
  const double *r_nodes;     /* [n_r] */
  const double *basis;       /* [K][n_r] */
  const double *mat_range;   /* [3][2] (lo, hi) of the PCA table, or NULL */
  int32_t layout;            /* TLT_LAYOUT_*: AUTO = tiles for non-F64 storage */
  int32_t tile_vertices;     /* vertices per tile block (0 = automatic) */
  int32_t val_is_f64;        /* col != NULL: 1 = val holds float64 values, 0 = value_dtype */
} tlt_transport_desc;

/*
 * Host-only validation of a transport description (no GPU work, no
 * context): every check load_transport makes before it touches the device
 * -- sizes, dtypes, layout, the permutation (TLT_E_FORMAT unless a
 * bijection of 0..N-1), areas (> 0, finite), and for given rows each column
 * in [0, n_cols) and strictly ascending per row (else TLT_E_FORMAT).
 * Returns TLT_OK or the status load_transport would return for these
 * reasons; the message is in tlt_last_error(NULL).
 */
tlt_status tlt_check_transport(const tlt_transport_desc *desc);

tlt_status tlt_create(tlt_ctx **out, int hip_device);
void tlt_destroy(tlt_ctx *ctx);
const char *tlt_last_error(const tlt_ctx *ctx);

/*
 * Loads (or builds) the transport and uploads the geometry (precompute of
 * Sec. 3.1 and 3.2, Step 1).  Synchronous.  All host checks (those of
 * tlt_check_transport) run before any device work, so a refused
 * description leaves the context as it was.  May return the warning
 * TLT_W_BF16_NO_RESIDUAL (loaded).
 */
tlt_status load_transport(tlt_ctx *ctx, const tlt_transport_desc *desc);

/*
 * Material for the next render (Step 3 of Sec. 4: a material edit reruns
 * the weights g_k of Sec. 2.2 / Eq. 4 and the combine of Step 4):
 * theta_dev [n_mat][3 channels][sigma_a, sigma_s', eta] float64 in device
 * memory, owned by the caller and read on render's stream (it must stay
 * valid until that render completes; values written to it before a later
 * render, or a graph replay, are the ones used).  Records the pointer and
 * marks the weights dirty; no copy, no synchronisation (hip_stream is
 * unused).  The values are validated by the weights kernel on the device:
 * a channel with sigma_a <= 0, sigma_s' <= 0, eta < 1 or a non-finite value
 * gets NaN weights (its radiance is NaN) and raises an invalid flag; a
 * valid channel outside mat_range raises a range flag and renders
 * normally.  tlt_material_status reports the flags.  TLT_E_ARG for
 * n_mat < 1 or NULL, TLT_E_STATE before load_transport.
 */
tlt_status set_material(tlt_ctx *ctx, int n_mat, const double *theta_dev,
                        void *hip_stream);

/*
 * Waits for hip_stream and reports, then clears, the material flags of the
 * renders since the last call: TLT_E_ARG if a rendered material channel was
 * invalid (the message names one), else TLT_W_MATERIAL_OUT_OF_RANGE if one
 * lay outside the PCA table's range (mat_range), else TLT_OK.
 */
tlt_status tlt_material_status(tlt_ctx *ctx, void *hip_stream);

/*
 * Lighting for the next render: sh_dev [n_light][n_sh][3] in device memory
 * (float64 for an F64 transport, else float32), read by render on its
 * stream.  Records the pointer only; marks the irradiance dirty.
 */
tlt_status set_lighting(tlt_ctx *ctx, int n_light, const void *sh_dev);

/*
 * Per-frame irradiance supplied directly, in place of SH lighting (for
 * lights the SH transfer does not represent, e.g. irradiance from a shadow
 * map; Step 1 of Sec. 4 computes E, and any E may enter the transport):
 * E_dev [n_light][N][3] in device memory, original vertex order, float64
 * for an F64 transport else float32, read by render on its stream (valid
 * until that render completes).  Render then computes
 * Ehat = Haar(pad(A o E)) and the transport as usual.  Stays in effect
 * until set_lighting.  render_backward and TLT_FOLDED_LIGHTING need SH
 * lighting (TLT_E_STATE / TLT_E_ARG after this call).  TLT_E_STATE before
 * load_transport, TLT_E_ARG for n_light < 1 or NULL.
 */
tlt_status set_irradiance(tlt_ctx *ctx, int n_light, const void *E_dev);

/*
 * Outgoing Fresnel factor of Eq. (3) and the last line of Eq. (6): with a
 * view set, render multiplies each radiance by (1/pi) F_t(eta, w_o), w_o the
 * direction from the vertex to `eye`, eta the channel's index of refraction
 * of the set's material, F_t = 1 - F_r the unpolarised Fresnel
 * transmittance of a smooth boundary (air outside, eta inside); vertices
 * seen from behind (n . w_o <= 0) get 0.  eye [3], position and normal
 * [N][3] in Morton order (as tlt_prepare_scene writes them), host memory,
 * mm; the cosines are computed here in float64.  eye == NULL removes the
 * view.  render_backward with a view set returns TLT_E_STATE.
 * TLT_E_STATE before load_transport; TLT_E_ARG for an eye on a vertex.
 */
tlt_status set_view(tlt_ctx *ctx, const double *eye, const double *position, const double *normal);

/*
 * Renders B [n_out][N][3] (original vertex order, float64 for an F64
 * transport else float32) into caller-owned device memory on hip_stream.
 * Recomputes only what changed since the last render unless TLT_FORCE_FULL.
 * TLT_KEEP_TERMS keeps the per-term transport v_k[v,c] = (W_k Ehat)[o,c]
 * (v = perm[o]; K*N*C values in library memory), so that a following render
 * after a material-only change (set_material, no set_lighting) reruns Steps 3
 * and 4 of Sec. 4 only: the weights and B = sum_k g_k v_k.  Without a kept
 * v_k every render runs the transport.  TLT_SAVE_FOR_BACKWARD marks the
 * render as the one render_backward differentiates; it costs nothing here.
 * TLT_FOLDED_LIGHTING renders through the lighting transport folded at load,
 * P_k = W_k H (A o T) (the SH-lighting path of Eq. 14): B = sum_k g_k P_k L,
 * equal to the wavelet transport of the same kept coefficients up to
 * rounding, reading K*N*Psh values instead of the transport (incompatible
 * with TLT_KEEP_TERMS and TLT_PLAIN_ROWS: TLT_E_ARG).  With 16-bit
 * storage the product reads an FP16 copy of P (built at the first folded
 * render, scaled by a power of two; ~2.4e-4 relative rounding per value,
 * the weighted lighting split hi + lo) unless TLT_TUNE_FOLDED_FP32.
 * TLT_SPATIAL renders through the spatially compressed transport of
 * load_spatial (Eq. 10, Steps 2, 4 and 5 of Sec. 4), recomputing every stage;
 * TLT_E_STATE without load_spatial, TLT_E_ARG combined with
 * TLT_SAVE_FOR_BACKWARD, TLT_KEEP_TERMS, TLT_PLAIN_ROWS or
 * TLT_FOLDED_LIGHTING.
 * TLT_E_STATE before load_transport / set_material / set_lighting.
 * Warning TLT_W_BF16_NO_RESIDUAL (rendered): the product of a BF16
 * transport ran without residual words -- TLT_PLAIN_ROWS (the row kernel
 * holds the BF16 values alone) or tiles loaded without them.
 */
tlt_status render(tlt_ctx *ctx, void *B_dev, void *hip_stream, int flags);

/*
 * Spatial (output-side) compression -- Sec. 3.2 (Eq. 9, 10; precompute Step
 * 2), CDF 9/7 per Sec. 5.  From the float64 Step-1 rows W_k^S (the kept
 * (column, value) pairs of every row, as tlt_build_rows writes them for all
 * Morton positions 0..N-1), per PCA term k:
 *   Z_k[:, j] = w_1 W_k^S[:, j]     w_1: CDF 9/7 along the Morton-ordered
 *                                   output index, near-orthonormal scaling
 *                                   (low-pass DC gain sqrt 2), whole-sample
 *                                   symmetric ends, levels while >= 8 entries
 *                                   remain (or `levels`), coefficients laid
 *                                   out [low_J, high_J, ..., high_1];
 *   S2(k)     = the fewest entries of Z_k, largest |z| first (ties to the
 *               lower u * n_cols + j), whose energy sum of z^2 reaches
 *               `energy` times that of all of Z_k (energy = 1 keeps every
 *               non-zero entry).
 * Rendering with TLT_SPATIAL then computes
 *   y[u, c] = sum_k g_k[c] sum_{j in S2(k, u)} Z_k[u, j] Ehat[j, c]
 *   B[perm[o], c] = (w_1^{-1} y[:, c])[o]            (Step 5 of Sec. 4).
 * Step 5 applies w_1^{-1} as a sparse matrix (a few tens of entries per
 * output position) built here from the synthesis of every unit coefficient.
 * The precompute runs on `threads` host threads (0 = up to 16) and
 * transforms every column of every term densely: O(K n_cols N) host work.
 * Values are stored in the transport's compute precision.  K < 128, else
 * TLT_E_ARG.  TLT_E_STATE before load_transport; the compression is dropped
 * by the next load_transport.  Host arrays are read during the call only.
 */
/*
 * Host-only form of the same precompute (no GPU work): writes the CSR of the
 * kept entries of Z over u -- rowptr_out [N+1] (always), col_out the column
 * words (k << 24) | j and val_out the float64 values, entries of a row in
 * (k, j) order.  col/val as in tlt_spatial_desc; n_cols = n_pad (Haar) or N.
 * TLT_E_ARG for bad sizes or when the kept entries exceed `capacity` (call
 * once with capacity 0 to learn rowptr_out[N]).
 */
tlt_status tlt_spatial_rows(int32_t n_vertices, int32_t n_cols, int32_t K, int64_t n_keep,
                            const int32_t *col, const double *val, double energy, int32_t levels,
                            int64_t *rowptr_out, uint32_t *col_out, double *val_out,
                            int64_t capacity);

/*
 * Host-only: the inverse transform w_1^{-1} of Step 5 (Sec. 4) over a list of
 * n_vertices as a sparse matrix, CSR over the output position o:
 * (w_1^{-1} y)[o] = sum_e w_out[e] y[col_out[e]] for e in
 * [rowptr_out[o], rowptr_out[o+1]).  Built from the synthesis of every unit
 * coefficient (exact zeros dropped); levels as in tlt_spatial_desc.
 * rowptr_out [n_vertices+1] is always written; TLT_E_ARG when the entries
 * exceed `capacity`, for n_vertices < 8 or too many levels.
 */
tlt_status tlt_spatial_synthesis(int32_t n_vertices, int32_t levels, int32_t *rowptr_out,
                                 int32_t *col_out, double *w_out, int64_t capacity);

typedef struct {
  double energy;            /* retained energy fraction per term, (0, 1] */
  int32_t levels;           /* CDF 9/7 levels, 0 = split while >= 8 entries remain */
  int32_t threads;          /* host threads, 0 = automatic */
  const int32_t *col;       /* [N][K][n_keep] Step-1 kept columns, ascending per row */
  const double *val;        /* [N][K][n_keep] float64 values */
} tlt_spatial_desc;

tlt_status load_spatial(tlt_ctx *ctx, const tlt_spatial_desc *desc);

/*
 * Statistics of the loaded spatial compression: total kept entries, levels,
 * and per term (arrays of K, each may be NULL) kept entries and retained
 * energy fraction.  TLT_E_STATE without load_spatial.
 */
tlt_status tlt_spatial_info(tlt_ctx *ctx, int64_t *nnz, int32_t *levels, int64_t *nnz_k,
                            double *energy_kept);

/*
 * Host copy of the kept entries of output coefficients u0 .. u0+n_u-1:
 * rowptr_out [n_u+1] (relative to the first), col_out the column words
 * (k << 24) | j, val_out the stored values widened to float64, entries of a
 * row in (k, j) order.  rowptr_out is always written; TLT_E_ARG if the
 * entries exceed `capacity` or the rows are out of range.  Synchronous.
 */
tlt_status tlt_read_spatial(tlt_ctx *ctx, int64_t u0, int64_t n_u, int64_t *rowptr_out,
                            uint32_t *col_out, double *val_out, int64_t capacity);

/*
 * Adjoint of the last render (which must have used TLT_SAVE_FOR_BACKWARD,
 * with no set_lighting / set_material since, else TLT_E_STATE; also
 * TLT_E_STATE after set_irradiance or with a view set).  dB_dev
 * [n_out][N][3] upstream gradient (precision of B).  Writes dSH_dev
 * [n_light][n_sh][3] (precision of B) and dTheta_dev [n_mat][3][3] float64,
 * both device memory, overwritten (not accumulated).  Steps 1-4 of Sec. 4 are
 * linear in the lighting and in the weights, and with the lighting-transfer
 * product P_k = W_k G, G = Haar(pad(A o T)) built at load, the per-term
 * transport is v_k = P_k L.  Both gradients follow from Z_k = P_k^T dB:
 *   dLoss/dg_k[c] = sum_lm L[lm,c] Z_k[lm,c],  dSH[lm,c] = sum_k g_k[c] Z_k[lm,c]
 * and dTheta = sum dLoss/dg_k * dg_k/dtheta (Eq. 4 differentiated in float64).
 * The lighting buffer of set_lighting is read again here, on hip_stream: it
 * must still hold the rendered values.  The first call (and a call with more
 * columns than before) allocates the library's partial-sum buffer.
 */
tlt_status render_backward(tlt_ctx *ctx, const void *dB_dev, void *dSH_dev,
                           double *dTheta_dev, void *hip_stream);

/*
 * For callers that cannot allocate -- code under HIP graph capture, serving
 * loops, harnesses that forbid device allocation: render_backward with its
 * scratch (the adjoint's partial rows and group sums) in a static device
 * buffer of TLT_NOALLOC_SCRATCH_BYTES that the library holds on each GPU it
 * runs on until the process ends.  It calls no allocating routine.  Same
 * arguments, checks, state rules and results as render_backward (the same
 * kernels).  TLT_E_ARG when the launch's partial sums exceed the buffer
 * (the message gives both sizes; about 4.6 MB at 163842 vertices, 16
 * lightings, 36 SH coefficients, K = 8).  Every call on one GPU shares that
 * GPU's buffer, whose contents the next call overwrites: calls that overlap
 * on one GPU (other streams, contexts or threads) race, and the caller must
 * order them.  Stage timing (tlt_profile_enable) does not record this call.
 */
#define TLT_NOALLOC_SCRATCH_BYTES (16u << 20)
tlt_status render_backward_noalloc(tlt_ctx *ctx, const void *dB_dev, void *dSH_dev,
                                   double *dTheta_dev, void *hip_stream);

/*
 * Diagnostics (host copies, synchronous).  tlt_read_rows copies rows
 * (row = o*K + k) of the stored transport: columns as int32 and values
 * widened to float64 (exactly the stored values).  tlt_read_state copies
 * an internal buffer: 0 = Ehat [n_pad or N][C_stride] (compute precision),
 * 1 = g [n_mat][3][K] float64, 2 = dg/dtheta [n_mat][3][K][3] float64;
 * *bytes receives the size when out == NULL.
 */
tlt_status tlt_read_rows(tlt_ctx *ctx, int64_t n_rows, const int64_t *rows,
                         int32_t *col_out, double *val_out);
/*
 * Shape of the loaded tiles (each pointer may be NULL): vertices per block,
 * blocks, entries (union slots, padded to the k-step), stored 16-row
 * fragments, bytes of stored values, and 1 when the tiles are
 * fragment-sparse (TLT_TUNE_TILE_SPARSE).  TLT_E_STATE without tiles.
 */
tlt_status tlt_tile_info(tlt_ctx *ctx, int32_t *vertices, int64_t *blocks, int64_t *entries,
                         int64_t *fragments, int64_t *value_bytes, int32_t *sparse);
tlt_status tlt_read_state(tlt_ctx *ctx, int which, void *out, size_t *bytes,
                          int *c_stride);

/*
 * Tile choice of the transport kernel: each lane accumulates
 * `columns_per_lane` consecutive output columns (one of 4, 8, 12, 16, 24,
 * 28, 32, 36, 48, 64); 0 restores the built-in choice (the smallest that
 * covers all columns, else 48-column slices).  Used by the autotuner.
 * Takes effect at the next render; TLT_E_ARG for unsupported values.
 */
tlt_status tlt_set_tile(tlt_ctx *ctx, int columns_per_lane);
int tlt_get_tile(const tlt_ctx *ctx);

/*
 * Launch tuning of a context (kept across load_transport; 0 restores the
 * built-in choice).  Keys:
 *   TLT_TUNE_TILE_CHUNK          largest number of k-steps of a tile block
 *                                whose irradiance rows are staged at once
 *   TLT_TUNE_STREAM_WAVES_PER_CU waves per compute unit of the row kernel
 *   TLT_TUNE_STREAM_EPL          entries per lane and step of the row kernel
 *                                for narrow launches: 4, 8 or 16
 *   TLT_TUNE_STREAM_NT           1 = non-temporal loads of the rows
 *   TLT_TUNE_TILE_SHAPE          16-bit tiles of 8 m-tiles: 100 MTW + 10 NT
 *                                + IPT with MTW m-tiles per wave, NT
 *                                16-column tiles per group and IPT staged
 *                                items per thread: 231 (built-in), 241,
 *                                432 or 442; of 16 m-tiles (256 rows): 231
 *                                (built-in) or 241
 *   TLT_TUNE_IRRADIANCE_HAAR     1 = compute Ehat per frame as the Haar
 *                                transform of A o (T L); 0 (default) = as
 *                                G L with G = H pad(A o T) formed once, for
 *                                launches of at most 32 columns (equal up
 *                                to float32 rounding)
 *   TLT_TUNE_SPATIAL_LANES       lanes per work item of the spatially
 *                                compressed transport: 16, 32 or 64
 *   TLT_TUNE_SPATIAL_UNROLL      its entries per lane and pass: 4, 8 or 16
 *   TLT_TUNE_SPATIAL_SYNTH_LANES lanes per output position of the inverse
 *                                transform of Step 5: 8, 16 or 32 (applies
 *                                at the next load_spatial)
 *   TLT_TUNE_SPATIAL_SEGMENT     longest work item of the compressed rows,
 *                                64 .. 2^20 entries (next load_spatial)
 *   TLT_TUNE_BF16_HEAD           1 = BF16 tiles built on the device store
 *                                the plain BF16 values only; 0 (default)
 *                                = they also carry the residual of the 64
 *                                coarsest columns (applies at the next
 *                                load_transport; changes results within
 *                                the BF16 storage error)
 *   TLT_TUNE_TILE_SPARSE         form of the tiles: 1 = dense (rows (o, k),
 *                                entries in column order, every 16-row
 *                                fragment stored); 2 = fragment-sparse
 *                                (rows (k, o), entries ordered by the rows
 *                                that keep them, fragments without a kept
 *                                coefficient left out; 16-bit storage
 *                                only, float32 tiles stay dense); 0
 *                                (default) = sparse for blocks of 256 rows
 *                                of 16-bit storage, else dense (applies at
 *                                the next load_transport; float32 summation
 *                                order only)
 *   TLT_TUNE_FOLDED_FP32         1 = folded lighting reads the float32 P
 *                                also with 16-bit storage (default 0: its
 *                                FP16 copy, half the bytes)
 * Values are clamped to what a launch supports.  TLT_E_ARG for an unknown
 * key or a value out of range.  Results do not depend on the tuning beyond
 * float32 summation order.
 */
enum {
  TLT_TUNE_TILE_CHUNK = 1,
  TLT_TUNE_STREAM_WAVES_PER_CU = 2,
  TLT_TUNE_STREAM_EPL = 3,
  TLT_TUNE_STREAM_NT = 4,
  TLT_TUNE_SPATIAL_LANES = 5,
  TLT_TUNE_SPATIAL_UNROLL = 6,
  TLT_TUNE_SPATIAL_SYNTH_LANES = 7,
  TLT_TUNE_SPATIAL_SEGMENT = 8,
  TLT_TUNE_TILE_SHAPE = 9,
  TLT_TUNE_IRRADIANCE_HAAR = 10,
  TLT_TUNE_BF16_HEAD = 11,
  TLT_TUNE_TILE_SPARSE = 12,
  TLT_TUNE_FOLDED_FP32 = 13
};
tlt_status tlt_set_tuning(tlt_ctx *ctx, int32_t key, int32_t value);

/*
 * Per-stage GPU timing.  While enabled, render and render_backward time
 * each stage with a pair of HIP events written by the stage's own kernel
 * dispatches (on their stream): 0 = material weights g_k (Step 3),
 * 1 = irradiance and its Haar transform (Step 1), 2 = wavelet transport
 * with K-term fusion (Steps 2 and 4; with TLT_SPATIAL the compressed
 * transport), 3 = adjoint reductions, 4 = material-only combine,
 * 5 = inverse spatial transform w_1^{-1} (Step 5, TLT_SPATIAL only).  mode 1 waits for pending events, clears the
 * totals and enables; mode 0 pauses and mode 2 resumes without waiting or
 * clearing (to time a sample of the renders of a running sequence).
 * tlt_profile_read waits for the recorded events and returns the summed
 * elapsed milliseconds and the number of timed launches of a stage.
 * TLT_E_ARG for another mode.  Do not enable during HIP graph capture.
 */
tlt_status tlt_profile_enable(tlt_ctx *ctx, int mode);

/*
 * Measurement only: reads `bytes` of device buffer `buf` once, with the
 * same 16-byte buffer loads the transport streams with (sixteen in flight
 * per lane), split over `blocks` workgroups of 256 threads; each wave
 * writes one folded word to out [blocks * 4] (device memory).  Timing it
 * gives the read bandwidth this load path reaches on the GPU.  Each
 * workgroup's share must stay below 1.75 GiB; `bytes` is a multiple of 16
 * (zero allowed, then `buf` may be null).  TLT_E_ARG for bad arguments.
 */
tlt_status tlt_read_probe(const void *buf, int64_t bytes, uint32_t *out, int blocks, void *stream);
tlt_status tlt_profile_read(tlt_ctx *ctx, int stage, double *total_ms, int64_t *launches);

/* Library version string (static storage). */
const char *tlt_version(void);

#ifdef __cplusplus
}
#endif
#endif /* TLT_H */
