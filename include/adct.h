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
 *   n          block length N in {8, 16, 32}.
 *   dtype      ADCT_U8: 8-bit grey levels, shifted by -128 before the
 *              transform and reconstructed as round(.) + 128 clipped to
 *              [0, 255].  ADCT_I16: signed 16-bit prediction residuals, not
 *              shifted, reconstruction saturated to int16.
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

/* Text of the last error on the calling thread ("" if none). */
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

/* JPEG zig-zag scan of an n x n block: host_out[k] = v * n + u of the k-th
 * scanned coefficient (n*n entries). */
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

/* Inverse of the compressed form: d_kept is int32 [tiles][r] as adct_compress
 * writes it (coefficients or, with qstep > 0, levels).  Writes the
 * reconstruction to d_dst; the result equals adct_compress's d_recon. */
ADCT_API int adct_decompress(int transform, int n, int r, int qstep, const int32_t* d_kept,
                             void* d_dst, int dtype, int batch, int height, int width,
                             int64_t pitch, int64_t image_stride, adct_stream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* ADCT_H_ */
