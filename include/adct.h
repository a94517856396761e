/*
 * adct.h -- C ABI of the MI355X (gfx950) library for the block-wise 2D
 * Chen-based approximate DCT of Tablada, da Silveira, Cintra and Bayer,
 * "DCT Approximations Based on Chen's Factorization".
 *
 * Every call takes plain host or device pointers and sizes.  Device buffers
 * are owned by the caller; the stateless calls below never allocate or free
 * device memory and only enqueue work on the caller's HIP stream (they return
 * as soon as the work is queued).  Calls return ADCT_OK or a negative status
 * and never abort; ``adct_last_error`` describes the last failure of the
 * calling thread.  Argument checks run before any HIP call, so a bad
 * argument is reported without touching the GPU.
 *
 * Terms used below
 *   transform  ADCT_T1: the sign-based approximation T~_N.  N = 8 is eq. 4
 *              (section 3); N = 16, 32 follow the Chen-JAM recursion of
 *              section 6.1.
 *              ADCT_T2: the round-based approximation T^_N (eq. 5 and
 *              section 6.1).
 *              ADCT_WHT, ADCT_SDCT, ADCT_HT: three of the 8-point transforms
 *              section 4 compares against (n = 8 only; ADCT_E_ARG otherwise).
 *              All three have add-only fast algorithms (24 additions, Table
 *              2) and exact integer inverses N T^-1, so every device call
 *              below computes them with the same kernels (the ragged-batch
 *              and serving calls take ADCT_T1 and ADCT_T2 only).
 *   n          block length N in {8, 16, 32, 64}.  The 64-point level of the
 *              recursion of section 6.1 takes ADCT_T1 / ADCT_T2, 8-bit images
 *              and zonal retention only (ADCT_E_ARG otherwise): its int32
 *              intermediates are exact for 8-bit input but not over the
 *              whole int16 range.
 *   dtype      ADCT_U8: 8-bit grey levels, shifted by -128 before the
 *              transform and reconstructed as round(.) + 128 clipped to
 *              [0, 255].  ADCT_I16: signed 16-bit prediction residuals, not
 *              shifted, reconstruction saturated to int16.  Every int16
 *              value is accepted: the int32 intermediates of all n, r and
 *              qstep stay exact over the whole int16 range.
 *   image set  ``batch`` images of ``height`` x ``width`` pixels (both
 *              multiples of n).  Row y of image i starts at element
 *              i * image_stride + y * pitch (strides in pixels, not bytes).
 *              Image start addresses and rows must be aligned to
 *              min(16, n * pixel size) bytes (ADCT_E_ALIGN otherwise).
 *   tile       the non-overlapping n x n block (ty, tx) of an image; tiles are
 *              numbered t = (i * (height/n) + ty) * (width/n) + tx.
 *   coefficient b[v][u] of B = T A T^T (section 5.1 with the separable
 *              form), v the vertical and u the horizontal frequency.  These
 *              are exact integers.
 *   r          number of retained coefficients: the first r positions of the
 *              JPEG zig-zag scan (section 5.1, generalised to N x N by
 *              anti-diagonals), 1 <= r <= n*n.
 *   qstep      0 selects zonal retention.  1..4096 selects the uniform
 *              quantiser of the orthonormal coefficients c = s_v s_u b with
 *              step qstep (section 3.1 lets the scale S be absorbed in the
 *              quantiser; the paper fixes no quantiser, see adct_quant_tables).
 *   stream     a hipStream_t passed as void*; NULL means the null stream.
 */
#ifndef ADCT_H_
#define ADCT_H_

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ADCT_API __attribute__((visibility("default")))

#define ADCT_T1 1
#define ADCT_T2 2
/* Comparison transforms of section 4 (Tables 1 and 2), n = 8 only: */
#define ADCT_WHT 3   /* Walsh-Hadamard, rows in sequency order  */
#define ADCT_SDCT 4  /* signed DCT, sign(C8)                    */
#define ADCT_HT 5    /* Hadamard, Sylvester's natural row order */
/* The exact DCT-II (section 2), the reference of section 5, n = 8, in float32:
 * adct_compress (zonal, d_kept NULL) and adct_compress_quality (no coding
 * gain) only; d_scaled receives its orthonormal coefficients. */
#define ADCT_DCT 6

#define ADCT_U8 0
#define ADCT_I16 1

#define ADCT_OK 0
#define ADCT_E_ARG (-1)     /* invalid id, n, r, qstep, dtype or null pointer */
#define ADCT_E_SHAPE (-2)   /* height/width not a multiple of n, bad strides   */
#define ADCT_E_ALIGN (-3)   /* misaligned image start or row pitch             */
#define ADCT_E_HIP (-4)     /* a HIP runtime call failed                        */
#define ADCT_E_BUDGET (-5)  /* a request exceeds a memory budget                */

typedef void* adct_stream_t;

/* Library version (integer, increases with every ABI change). */
ADCT_API int adct_version(void);

/* Text of the last error on the calling thread ("" if none); library
 * bookkeeping, no operation of the paper.  The string is owned by the
 * library and valid until the thread's next call. */
ADCT_API const char* adct_last_error(void);

/* ----------------------------------------------------------------------
 * Host-side queries.  No GPU needed.  They report what the library's own
 * kernels compute, derived on the host from the same add-only butterflies.
 * ---------------------------------------------------------------------- */

/* n*n int32 row-major matrix into host_out.  inverse = 0: T_N (eqs. 4/5 and
 * the recursion of section 6.1), obtained by running the forward butterfly on
 * unit vectors.  inverse = 1: U_N = N * T_N^-1 (eqs. 6/7 and the inverse
 * factorization of section 6.1), from the inverse butterfly.  */
ADCT_API int adct_get_matrix(int transform, int n, int inverse, int32_t* host_out);

/* Section 4.1's assessment measures of the transform (host-side, float64):
 * *eps = pi ||C_N - S' T_N||_F^2, the total error energy against the
 * orthonormal DCT-II C_N (Table 1), and *delta = 1 - ||diag(M)||^2 / ||M||_F^2
 * for M = T_N T_N^T, the deviation from diagonality (section 3.1).  Either
 * pointer may be NULL.  Both are 0 for ADCT_DCT. */
ADCT_API int adct_transform_measures(int transform, int n, double* eps, double* delta);

/* The zig-zag scan of section 5.1 (the JPEG rule, generalised to n x n by
 * anti-diagonals): host_out[k] = v * n + u of the k-th scanned coefficient
 * (n*n entries, caller-owned host memory).  ADCT_E_ARG for a bad n or a null
 * pointer. */
ADCT_API int adct_zigzag(int n, int32_t* host_out);

/* s_k = 1 / sqrt((T_N T_N^T)_kk), the diagonal of S' (section 3.1), in double
 * precision (n entries). */
ADCT_API int adct_scale_vector(int transform, int n, double* host_out);

/* The fixed-point uniform quantiser used when qstep > 0 (n*n entries each,
 * row-major in (v, u)):
 *   g_vu = qstep * sqrt(d_v d_u), d = diag(T T^T)
 *   mq_vu = round(2^24 / g_vu)       level = sign(b) * ((|b| * mq + 2^23) >> 24)
 *   dq_vu = round(2 * g_vu)          dequantised coefficient = level * dq
 * with round() half away from zero (section 3); the dequantised values carry
 * one fractional bit, so the reconstruction divides by 2 N^2. */
ADCT_API int adct_quant_tables(int transform, int n, int qstep, int32_t* mq, int32_t* dq);

/* ----------------------------------------------------------------------
 * Device entry points (asynchronous on ``stream``).
 * ---------------------------------------------------------------------- */

/* Forward 2D transform of every tile (section 5.1): d_coef receives all n*n
 * coefficients of tile t at d_coef[t * n*n + v * n + u] (int32, natural
 * order, device memory, batch * height * width entries). */
ADCT_API int adct_fwd2d(int transform, int n, const void* d_src, int dtype, int batch,
                        int height, int width, int64_t pitch, int64_t image_stride,
                        int32_t* d_coef, adct_stream_t stream);

/* Inverse 2D transform (eqs. 6/7, section 6.1) of natural-order coefficients
 * laid out as adct_fwd2d writes them.  Only the first r zig-zag positions of
 * each tile are used (r = n*n uses all).  qstep > 0: d_coef holds quantiser
 * levels, which are dequantised first.  The result is written to d_dst with
 * the given geometry.  Exact for coefficients produced by adct_fwd2d or
 * adct_compress; other inputs may overflow 32-bit arithmetic. */
ADCT_API int adct_inv2d(int transform, int n, int r, int qstep, const int32_t* d_coef,
                        void* d_dst, int dtype, int batch, int height, int width,
                        int64_t pitch, int64_t image_stride, adct_stream_t stream);

/* The fused pipeline of section 5.1 in one pass: forward transform, zonal
 * retention of the first r zig-zag coefficients (or quantisation when
 * qstep > 0), inverse transform, rounding and clipping, error energy.
 * Every output pointer may be NULL (that output is skipped):
 *   d_kept   int32 [tiles][r]: the retained coefficients in zig-zag order
 *            (quantiser levels when qstep > 0);
 *   d_scaled float [tiles][r]: s_v s_u b_vu of the same positions, the
 *            coefficients of the near-orthogonal C = S' T (section 3.1);
 *   d_recon  reconstruction, same dtype and geometry as d_src;
 *   d_sse    uint64 [batch]: sum of squared reconstruction errors of each
 *            image, ADDED to the existing values (the caller zeroes them).
 * PSNR follows as 10 log10(255^2 * H * W / sse). */
ADCT_API int adct_compress(int transform, int n, int r, int qstep, const void* d_src, int dtype,
                           int batch, int height, int width, int64_t pitch,
                           int64_t image_stride, int32_t* d_kept, float* d_scaled,
                           void* d_recon, uint64_t* d_sse, adct_stream_t stream);

/* Inverse of the compressed form (section 5.1 with the exact inverse of
 * eqs. 6/7 and section 6.1): d_kept is int32 [tiles][r] as adct_compress
 * writes it (coefficients or, with qstep > 0, levels).  Writes the
 * reconstruction to d_dst; the result equals adct_compress's d_recon. */
ADCT_API int adct_decompress(int transform, int n, int r, int qstep, const int32_t* d_kept,
                             void* d_dst, int dtype, int batch, int height, int width,
                             int64_t pitch, int64_t image_stride, adct_stream_t stream);

/* The fused compress of adct_compress for n = 8, ADCT_U8 and zonal
 * retention (qstep 0), computed on the int8 matrix cores instead of the
 * butterflies: vec(B) = (T (x) T) vec(A - 128) and the exact inverse
 * vec(X) = (U (x) U) vec(B~) with U = 8 T^-1 (section 3, eqs. 4-7), both
 * Kronecker products having entries in {0, +-1, +-2, +-4}.  Arguments,
 * layouts and outputs are those of adct_compress (outputs bit-identical);
 * image rows must be 8-byte aligned. */
ADCT_API int adct_compress_mfma(int transform, int r, const void* d_src, int batch, int height,
                                int width, int64_t pitch, int64_t image_stride, int32_t* d_kept,
                                float* d_scaled, void* d_recon, uint64_t* d_sse,
                                adct_stream_t stream);

/* ----------------------------------------------------------------------
 * Quality measures: PSNR (section 5.1) and the unified coding gain
 * (section 4.1), in float32.
 * ---------------------------------------------------------------------- */

/* g_k of the coding gain: the rows of C^-1 (as section 4.1 words it) or its
 * columns (the synthesis basis).  Both agree for orthogonal transforms. */
#define ADCT_BASIS_ROWS 0
#define ADCT_BASIS_COLS 1

/* uint64 words of one moment record of block length n. */
#define ADCT_MOMENT_WORDS(n) (3 * (n) * (n) + 4)

/* SSIM of section 5.1 (the index of Wang et al., which the paper cites):
 * d_ssim[i] (float32) is the mean over every full 11 x 11 window of image i
 * of (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2)),
 * with Gaussian-weighted (sigma 1.5) means, variances and covariance of the
 * 8-bit images d_x and d_y (same geometry: batch images of height x width
 * >= 11 x 11, row pitch and image stride in bytes), C1 = (0.01 * 255)^2,
 * C2 = (0.03 * 255)^2.  d_work: batch float64 accumulators of caller-owned
 * device memory, 8-byte aligned, zeroed by the call. */
ADCT_API int adct_ssim(const void* d_x, const void* d_y, int batch, int height, int width,
                       int64_t pitch, int64_t image_stride, double* d_work, float* d_ssim,
                       adct_stream_t stream);

/* Absolute percentage error of section 5.1: d_ape[i] = 100 |d_value[i] -
 * d_reference[i]| / |d_reference[i]| (float32 device arrays of count entries;
 * the reference is the exact DCT's measure for the same image). */
ADCT_API int adct_ape(int count, const float* d_value, const float* d_reference, float* d_ape,
                      adct_stream_t stream);

/* PSNR of section 5.1 from error energies: d_psnr[i] = 10 log10(255^2 *
 * pixels / d_sse[i]) in float32, +inf where d_sse[i] = 0 (device arrays of
 * count entries; pixels >= 1 is the pixel count of every image).  count = 0
 * is a no-op. */
ADCT_API int adct_psnr(int count, int64_t pixels, const uint64_t* d_sse, float* d_psnr,
                       adct_stream_t stream);

/* Moments of the coefficients b[v][u] of B = T A T^T over the tiles of each
 * image (section 5.1), and of its pixels a (8-bit input shifted by -128),
 * ADDED to the record of that image (the caller zeroes the records first;
 * records of several calls may be accumulated).  d_moments holds batch
 * records of ADCT_MOMENT_WORDS(n) uint64 words, 8-byte aligned device memory:
 *   [p]            sum over tiles of b_p, as two's complement int64,
 *                  p = v * n + u;
 *   [n*n + p]      sum over tiles of (b_p^2 mod 2^32);
 *   [2*n*n + p]    sum over tiles of floor(b_p^2 / 2^32), so that the sum of
 *                  b_p^2 is word[2n^2 + p] * 2^32 + word[n^2 + p];
 *   [3*n*n]        tiles;   [3*n*n + 1] pixels;
 *   [3*n*n + 2]    sum of a (two's complement int64);  [3*n*n + 3] sum of a^2.
 * Every sum is exact for every input of up to 2^32 tiles per image.  Image
 * set arguments as for adct_fwd2d.  Only d_moments is written. */
ADCT_API int adct_moments(int transform, int n, const void* d_src, int dtype, int batch,
                          int height, int width, int64_t pitch, int64_t image_stride,
                          uint64_t* d_moments, adct_stream_t stream);

/* Measured 2D coding gain (dB) of each of count moment records (as
 * adct_moments writes them, same transform and n): the unified coding gain of
 * section 4.1 for the separable transform C (x) C, C = S' T, with A_vu the
 * variance of the orthonormal coefficient s_v s_u b_vu over the tiles divided
 * by the pixel variance, and B_v B_u the squared norm of the synthesis vector
 * g_v g_u^T (basis: ADCT_BASIS_ROWS or ADCT_BASIS_COLS):
 *   d_cg[i] = -10 / n^2 * sum_vu log10(A_vu B_v B_u).
 * +inf when a coefficient has zero variance, NaN when the pixels have zero
 * variance or the record is empty.  float32 output, device arrays. */
ADCT_API int adct_coding_gain(int transform, int n, int basis, int count,
                              const uint64_t* d_moments, float* d_cg, adct_stream_t stream);

/* adct_compress plus the quality measures of each image in one call: the
 * fused pipeline (outputs d_kept, d_scaled, d_recon as in adct_compress, each
 * nullable), then d_psnr[i] (float32 PSNR of image i, section 5.1, nullable)
 * and d_cg[i] (its measured 2D coding gain, as adct_coding_gain with the
 * given basis, section 4.1; nullable).  The error energies and moment records
 * this needs live in the caller's device workspace d_work (8-byte aligned,
 * work_bytes >= adct_compress_quality_workspace(n, batch, d_cg != NULL));
 * the call zeroes them itself, and their contents after the call are
 * unspecified.  ADCT_E_BUDGET when the workspace is too small.  Other
 * arguments and errors as for adct_compress. */
ADCT_API int adct_compress_quality(int transform, int n, int r, int qstep, const void* d_src,
                                   int dtype, int batch, int height, int width, int64_t pitch,
                                   int64_t image_stride, int32_t* d_kept, float* d_scaled,
                                   void* d_recon, float* d_psnr, float* d_cg, int basis,
                                   void* d_work, int64_t work_bytes, adct_stream_t stream);

/* adct_compress_quality for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same arguments without the workspace, the same outputs.
 * The error energies and moment records go to a fixed scratch array of
 * 2^19 64-bit words (4 MiB) that the library holds on every GPU it runs on
 * until the process ends, so batch * (1 + (d_cg != NULL ? ADCT_MOMENT_WORDS(n)
 * : 0)) must not exceed 524288 (ADCT_E_BUDGET otherwise, before any GPU
 * work).  The call allocates and frees no device memory.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams,
 * other threads) race and their results are undefined.  Call it with the
 * device of `stream` current. */
ADCT_API int adct_compress_quality_noalloc(int transform, int n, int r, int qstep,
                                           const void* d_src, int dtype, int batch, int height,
                                           int width, int64_t pitch, int64_t image_stride,
                                           int32_t* d_kept, float* d_scaled, void* d_recon,
                                           float* d_psnr, float* d_cg, int basis,
                                           adct_stream_t stream);

/* Bytes of the workspace adct_compress_quality needs: 8 * batch * (1 +
 * (with_coding_gain ? ADCT_MOMENT_WORDS(n) : 0)); a negative status for a bad
 * n or batch.  Host-side. */
ADCT_API int64_t adct_compress_quality_workspace(int n, int batch, int with_coding_gain);

/* Coding gain (dB) of C = S' T under the first-order Markov model of section
 * 4.1, R_x[m][n] = rho^|m - n|, for count correlation values d_rho[i] in
 * [0, 1) (device float32): d_cg[i] = -10 / n * sum_k log10(A_k B_k) with
 * A_k = h_k R_x h_k^T, h_k row k of C, and B_k the squared norm of row or
 * column k of C^-1 (basis).  d_cg_klt[i] receives the KLT's gain for the same
 * rho, -10 / n * sum log10 lambda(R_x) = -10 (n-1)/n log10(1 - rho^2).
 * Either output may be NULL.  float32, device arrays. */
ADCT_API int adct_coding_gain_ar1(int transform, int n, int basis, int count,
                                  const float* d_rho, float* d_cg, float* d_cg_klt,
                                  adct_stream_t stream);

/* ----------------------------------------------------------------------
 * Measurement aid (no operation of the paper): the streaming ceiling of the
 * HBM that the fused kernels' bandwidth is compared with.  pattern 0 reads
 * `bytes` from d_src (d_dst receives at most one word, only for a pattern no
 * zero-filled input produces; pass a zero-filled d_src), 1 writes `bytes` of
 * zeros to d_dst, 2 copies `bytes` from d_src to d_dst; 16-byte non-temporal
 * accesses, `blocks` workgroups of 256 threads in grid-stride order with
 * `unroll` (1, 2, 4 or 8) independent loads in flight per thread.  Patterns
 * 3, 4 and 5 are the same read, write and copy with each workgroup walking
 * one contiguous chunk of the buffer.  bytes a multiple of 16, buffers
 * 16-byte aligned.
 * ---------------------------------------------------------------------- */
ADCT_API int adct_stream_ceiling(int pattern, void* d_dst, const void* d_src, int64_t bytes,
                                 int blocks, int unroll, adct_stream_t stream);

/* ----------------------------------------------------------------------
 * Ragged batches: many images of different sizes, each partitioned into
 * square transform units (TUs) of 8, 16 or 32 pixels (an HEVC-style quadtree;
 * section 6 embeds the 16- and 32-point transforms in such a coder).
 *
 * A plan sorts the TUs into buckets of one size, transform and step (and, for
 * 8x8 TUs, r <= 32 or not), orders each bucket by image and cuts it into work
 * items of one image each, sized to one workgroup.  It owns that device work
 * list until adct_batch_destroy.  adct_batch_run processes every TU with the
 * fused pipeline of adct_compress: one launch per bucket over all images, a
 * replay of that launch sequence captured in a HIP graph, or (for
 * comparison) one launch per image and bucket.  A plan is not thread-safe;
 * concurrent runs of one plan race on its graph cache.
 * ---------------------------------------------------------------------- */

typedef struct {
  int64_t src_offset; /* pixel offset of the image's pixel (0, 0) in d_src      */
  int64_t dst_offset; /* pixel offset of its reconstruction in d_dst            */
  int32_t height;     /* pixels, multiple of 8                                  */
  int32_t width;      /* pixels, multiple of 8                                  */
  int32_t pitch;      /* pixels between rows (same in d_src and d_dst), >= width */
  int32_t transform;  /* ADCT_T1 or ADCT_T2                                     */
  int32_t r;          /* zig-zag prefix kept per TU (a TU of size n keeps min(r, n*n)) */
  int32_t qstep;      /* 0 (zonal) or 1..4096 (quantiser, see adct_quant_tables) */
} adct_image_desc_t;

typedef struct {
  int32_t image; /* index into the image table                  */
  int32_t x;     /* left column of the TU, multiple of n          */
  int32_t y;     /* top row of the TU, multiple of n              */
  int32_t n;     /* 8, 16 or 32; the TU must lie inside the image */
} adct_tu_desc_t;

typedef struct adct_batch adct_batch_t;

#define ADCT_RUN_BATCHED 0   /* one launch per bucket, covering every image      */
#define ADCT_RUN_GRAPH 1     /* replay of the tuned sequence (per-bucket or     */
                             /* unified) captured in a HIP graph                */
#define ADCT_RUN_PER_IMAGE 2 /* one launch per image and bucket (baseline)       */
#define ADCT_RUN_UNIFIED 3   /* one launch per quantiser class covering every     */
                             /* bucket, items of all sizes in image/position order */
/* The zonal class of the unified launch runs every TU size one tile row per
 * thread when none of its 16x16 / 32x32 TUs keeps more than r = 36 (the
 * first 8 anti-diagonals): only 8 rows or columns of a tile then cross LDS,
 * and the launch fits more workgroups per compute unit (adct_batch_info
 * reports which form a plan uses). */

/* Build a plan (host arrays in, device work list out; allocates device memory
 * and synchronises the device).  dtype is ADCT_U8 or ADCT_I16 for every
 * image.  Image offsets and pitches must be multiples of 16 bytes.  The
 * retained coefficients of all TUs are packed into one array of *kept_words
 * words: TU t owns words [tu_kept_offset[t], + min(r, n*n)) in zig-zag order
 * (tu_kept_offset may be NULL).  TUs may be given in any order; TUs of one
 * image must not overlap (ADCT_E_SHAPE otherwise, like a TU outside its
 * image or not aligned to its size). */
ADCT_API int adct_batch_create(const adct_image_desc_t* images, int n_images,
                               const adct_tu_desc_t* tus, int64_t n_tus, int dtype,
                               int64_t* tu_kept_offset, int64_t* kept_words,
                               adct_batch_t** plan);

/* Free a plan and its device work lists (bookkeeping; waits for nothing, so
 * the caller must not destroy a plan whose runs are still queued). */
ADCT_API int adct_batch_destroy(adct_batch_t* plan);

/* Run the plan: every TU goes through the pipeline of adct_compress (section
 * 5.1 with the transforms of eqs. 4/5 and section 6.1).  d_src / d_dst are
 * pixel arenas addressed by the image descriptors (16-byte aligned);
 * d_kept/d_scaled hold kept_words int32/float words; d_sse and d_psnr hold one
 * uint64/float per image.  d_sse is overwritten with the error energy of this
 * run and d_psnr receives 10 log10(255^2 H W / sse) (+inf when sse = 0) in
 * single precision.  Any output may be NULL, except that d_psnr needs d_sse.
 * mode is one of ADCT_RUN_*; ADCT_RUN_GRAPH needs a non-null stream and re-
 * captures only when a buffer or the stream changes. */
ADCT_API int adct_batch_run(adct_batch_t* plan, const void* d_src, void* d_dst, int32_t* d_kept,
                            float* d_scaled, uint64_t* d_sse, float* d_psnr, int mode,
                            adct_stream_t stream);

/* Launch shape of the plan and its tuning (no operation of the paper).
 * Workgroup sizes:
 * bs8 threads (64 or 256) for 8x8 buckets, bs_jam (128 or
 * 256) for 16x16 and 32x32 buckets; a workgroup processes bs8 8x8 TUs or
 * bs_jam / n larger TUs (the unified launch always uses 256).
 * adct_batch_tune times both candidates of every bucket on the given buffers
 * (synchronising the stream), keeps the fastest and writes it to
 * chosen[bucket] (chosen may be NULL); it then times the tuned per-bucket
 * sequence against the unified launch and keeps the faster as the sequence
 * ADCT_RUN_GRAPH captures (the unified launch until a plan is tuned).  For
 * the row-per-thread unified launch it also times the tile groups per item of
 * 8x8 and 16x16 TUs (1, 2 or 4) and a persistent grid (4 or 8 resident
 * workgroups per compute unit walking XCD slices of the items) against one
 * workgroup per item, and keeps the fastest.  When
 * the environment variable ADCT_TUNE_CACHE names a file, choices are cached
 * there keyed by device architecture and plan shape and reused by later
 * plans. */
ADCT_API int adct_batch_set_shape(adct_batch_t* plan, int bs8, int bs_jam);
/* The row-per-thread unified launch's shape (what adct_batch_tune searches):
 * tile groups per work item for 8x8 and for 16x16 TUs (1, 2, 4 or 8; a 32x32
 * item holds one group), and persistent = 1 for a grid of wgs_per_cu (1..16)
 * workgroups per compute unit that walk the items instead of one workgroup
 * per item.  Rebuilds the plan's unified work list (synchronises). */
ADCT_API int adct_batch_set_small_shape(adct_batch_t* plan, int groups8, int groups16,
                                        int persistent, int wgs_per_cu);
ADCT_API int adct_batch_tune(adct_batch_t* plan, const void* d_src, void* d_dst, int32_t* d_kept,
                             float* d_scaled, uint64_t* d_sse, adct_stream_t stream, int* chosen);

/* Work-list statistics (bookkeeping): out[0..13] = images, TUs, work items,
 * items of size 8, 16 and 32, buckets, compute units of the device, items
 * of the unified launches, 1 when the zonal unified launch is the
 * row-per-thread form for kept bounds <= 8 (else 0), that form's tile groups
 * per item for 8x8 and for 16x16 TUs, 1 when it runs as a persistent grid,
 * and the persistent grid's workgroups per compute unit. */
ADCT_API int adct_batch_info(const adct_batch_t* plan, int64_t* out);

/* ----------------------------------------------------------------------
 * Serving: continuous batching of independent compress requests.
 *
 * Each request is one image compressed with the fused pipeline (section 5.1;
 * eqs. 4/5 and section 6.1) of
 * adct_compress (its own transform, n, r, qstep and dtype).  A server admits
 * requests against an HBM budget, queues them, and launches whatever is
 * queued as one batch whenever one of its max_inflight batch slots is free:
 * one launch per (transform, n, dtype, quantiser, r class) covering every
 * request of that class in the batch.  Requests that arrive while batches
 * run join the next batch, so the batch size follows the load.  Each slot
 * has its own stream, ordered after the caller's stream at every flush, so
 * consecutive batches run side by side on the device and may complete out
 * of order.
 *
 * Memory.  The server owns a device arena of budget_bytes for the outputs
 * (reconstruction with the request's pitch, retained coefficients, optional
 * scaled coefficients), allocated at the first flush.  A request is charged
 * its input plus its outputs; adct_server_submit returns ADCT_E_BUDGET when
 * the charge does not fit next to the requests in flight (retry after a
 * poll), or when it exceeds the whole budget.  The arena is a ring: a
 * block is reused once every older block has been released.
 *
 * Time.  done_ms and adct_server_clock_ms use one clock: milliseconds of the
 * host's steady clock since the server was created.  A batch's completion
 * time is read from a HIP event recorded after its last operation, aligned
 * to the host clock once at the first flush.
 *
 * A server is not thread-safe: one host thread drives it.
 * ---------------------------------------------------------------------- */

typedef struct adct_server adct_server_t;

typedef struct {
  const void* d_src;   /* device pixels, valid until the request completes       */
  void* h_kept;        /* NULL, or host memory receiving the tiles*r kept words  */
  void* h_scaled;      /* NULL, or host memory receiving tiles*r scaled floats   */
  void* h_recon;       /* NULL, or host memory receiving height*pitch pixels     */
  int64_t pitch;       /* pixels between rows, >= width                         */
  int64_t tag;         /* caller's identifier, echoed in the completion          */
  int32_t transform;   /* ADCT_T1 or ADCT_T2                                     */
  int32_t n;           /* 8, 16 or 32                                            */
  int32_t r;           /* 1 <= r <= n*n                                          */
  int32_t qstep;       /* 0 (zonal) or 1..4096                                   */
  int32_t dtype;       /* ADCT_U8 or ADCT_I16                                    */
  int32_t height;      /* multiple of n                                          */
  int32_t width;       /* multiple of n                                          */
  int32_t want_scaled; /* nonzero: also compute the float32 scaled coefficients  */
                       /* (h_scaled needs want_scaled)                           */
} adct_request_t;

typedef struct {
  int64_t tag;             /* the request's tag                                  */
  int64_t batch;           /* sequence number of the batch it ran in (0, 1, ...) */
  uint64_t sse;            /* error energy of its reconstruction                 */
  double done_ms;          /* completion time on the server clock                */
  double launch_ms;        /* host time (server clock) of the flush that launched */
                           /*   the request's batch                               */
  const int32_t* d_kept;   /* outputs in the arena, valid until the next poll:   */
  const float* d_scaled;   /*   kept [tiles][r] (zig-zag order), scaled (or NULL), */
  const void* d_recon;     /*   reconstruction (height rows of pitch pixels)     */
} adct_completion_t;

/* Create a server (host state only; no HIP call).  budget_bytes > 0,
 * 1 <= max_inflight <= 8 batch slots, 1 <= max_batch <= 4096 requests per
 * batch; work is enqueued on stream. */
ADCT_API int adct_server_create(int64_t budget_bytes, int max_inflight, int max_batch,
                                adct_stream_t stream, adct_server_t** server);

/* Wait for every launched batch, then free the server and its arena
 * (bookkeeping). */
ADCT_API int adct_server_destroy(adct_server_t* server);

/* Validate and admit one request (admission bookkeeping, host only; the
 * request is copied, its buffers stay caller-owned).  ADCT_OK: queued.
 * ADCT_E_BUDGET: not admitted now (or never, if it exceeds the budget). */
ADCT_API int adct_server_submit(adct_server_t* server, const adct_request_t* request);

/* Launch the queued requests (at most max_batch, oldest first) as one batch
 * if a batch slot is free: each request runs the pipeline of adct_compress
 * (section 5.1); *launched receives the number of requests
 * launched (0 when nothing is queued or every slot is busy). */
ADCT_API int adct_server_flush(adct_server_t* server, int* launched);

/* Report completed batches (bookkeeping; in launch order among those
 * complete) as long as their requests fit in out[0 .. max_out) (max_out must
 * be at least max_batch).  wait != 0 blocks
 * until every launched batch has completed.  Arena space of the batches
 * reported by the previous poll is released first. */
ADCT_API int adct_server_poll(adct_server_t* server, int wait, adct_completion_t* out,
                              int max_out, int* n_out);

/* Statistics (bookkeeping): out[0..7] = submitted, completed, batches
 * launched, queued, in flight, bytes charged, largest batch, ADCT_E_BUDGET
 * refusals. */
ADCT_API int adct_server_stats(const adct_server_t* server, int64_t* out);

/* Milliseconds on the server clock (bookkeeping; 0 for a null server). */
ADCT_API double adct_server_clock_ms(const adct_server_t* server);

/* Replay an arrival trace in real time on the calling thread: request i
 * arrives arrival_ms[i] milliseconds after the start (non-decreasing), is
 * admitted in arrival order (waiting while the budget is full), batched and
 * launched through the pipeline of adct_compress (section 5.1); the call
 * returns when every request has completed.
 * latency_ms[i] = completion - arrival, batch_of[i] = its batch, sse[i] = its
 * error energy, launch_ms[i] = host time of the flush that launched it,
 * milliseconds after the start (launch_ms - arrival is the time it waited on
 * the host, latency - that the time on the device); any of the four may be
 * NULL.  A request that fails validation gets latency and launch time NaN
 * and batch -1.  The server must be idle. */
ADCT_API int adct_server_run_trace(adct_server_t* server, const adct_request_t* requests,
                                   const double* arrival_ms, int64_t n, double* latency_ms,
                                   int64_t* batch_of, uint64_t* sse, double* launch_ms);

#ifdef __cplusplus
}
#endif

#endif /* ADCT_H_ */
