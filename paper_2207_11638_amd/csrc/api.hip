// C ABI: argument checks, constant tables and kernel dispatch.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/adct.h"
#include "adct_internal.hpp"

namespace adct {
namespace {

thread_local std::string g_last_error;

int fail(int status, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int status, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return status;
}

int ok() {
  g_last_error.clear();
  return ADCT_OK;
}

bool valid_kind(int t) { return t >= ADCT_T1 && t <= ADCT_DCT; }
// the comparison transforms of section 4 are 8-point transforms
bool valid_kind_n(int t, int n) { return t == ADCT_T1 || t == ADCT_T2 || n == 8; }
bool valid_n(int n) { return n == 8 || n == 16 || n == 32 || n == 64; }

// Apply the forward (inverse = false) or inverse butterfly of (kind, n) to a
// vector on the host.
void apply_1d(int kind, int n, bool inverse, int* v) {
#define ADCT_APPLY(K, NN)                             \
  do {                                                \
    int tmp[NN];                                      \
    for (int i = 0; i < NN; ++i) tmp[i] = v[i];       \
    if (inverse) invN<K, NN>(tmp); else fwdN<K, NN>(tmp); \
    for (int i = 0; i < NN; ++i) v[i] = tmp[i];       \
  } while (0)
  if (kind == KIND_WHT) {
    ADCT_APPLY(KIND_WHT, 8);
  } else if (kind == KIND_SDCT) {
    ADCT_APPLY(KIND_SDCT, 8);
  } else if (kind == KIND_HT) {
    ADCT_APPLY(KIND_HT, 8);
  } else if (kind == KIND_SIGN) {
    if (n == 8) ADCT_APPLY(KIND_SIGN, 8);
    else if (n == 16) ADCT_APPLY(KIND_SIGN, 16);
    else if (n == 32) ADCT_APPLY(KIND_SIGN, 32);
    else ADCT_APPLY(KIND_SIGN, 64);
  } else {
    if (n == 8) ADCT_APPLY(KIND_ROUND, 8);
    else if (n == 16) ADCT_APPLY(KIND_ROUND, 16);
    else if (n == 32) ADCT_APPLY(KIND_ROUND, 32);
    else ADCT_APPLY(KIND_ROUND, 64);
  }
#undef ADCT_APPLY
}

// Column j of the operator = operator applied to e_j.
void operator_matrix(int kind, int n, bool inverse, std::vector<int>& m) {
  m.assign(n * n, 0);
  std::vector<int> e(n);
  for (int j = 0; j < n; ++j) {
    std::fill(e.begin(), e.end(), 0);
    e[j] = 1;
    apply_1d(kind, n, inverse, e.data());
    for (int i = 0; i < n; ++i) m[i * n + j] = e[i];
  }
}

// diag(T T^T) from the forward butterfly.
void diag_ttt(int kind, int n, std::vector<int64_t>& d) {
  std::vector<int> t;
  operator_matrix(kind, n, false, t);
  d.assign(n, 0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) d[i] += static_cast<int64_t>(t[i * n + j]) * t[i * n + j];
}

double round_half_away(double x) { return x < 0 ? -floor(-x + 0.5) : floor(x + 0.5); }

struct TableSet {
  Tables t;
  std::vector<int32_t> mq_full, dq_full;
};

// Class tables: the distinct diagonal values (at most four) index the scale
// and quantiser tables.
template <int KIND, int N>
void classes_of(std::vector<int64_t>& vals, std::vector<int>& cls) {
  const RowClasses<N> rc = row_classes<KIND, N>();   // the kernels use the same numbering
  vals.assign(rc.value, rc.value + rc.count);
  cls.assign(rc.cls, rc.cls + N);
}

int build_tables(int kind, int n, int qstep, TableSet& out) {
  std::vector<int64_t> vals;
  std::vector<int> cls;
  if (kind == KIND_WHT) {
    classes_of<KIND_WHT, 8>(vals, cls);
  } else if (kind == KIND_SDCT) {
    classes_of<KIND_SDCT, 8>(vals, cls);
  } else if (kind == KIND_HT) {
    classes_of<KIND_HT, 8>(vals, cls);
  } else if (kind == KIND_SIGN) {
    if (n == 8) classes_of<KIND_SIGN, 8>(vals, cls);
    else if (n == 16) classes_of<KIND_SIGN, 16>(vals, cls);
    else if (n == 32) classes_of<KIND_SIGN, 32>(vals, cls);
    else classes_of<KIND_SIGN, 64>(vals, cls);
  } else {
    if (n == 8) classes_of<KIND_ROUND, 8>(vals, cls);
    else if (n == 16) classes_of<KIND_ROUND, 16>(vals, cls);
    else if (n == 32) classes_of<KIND_ROUND, 32>(vals, cls);
    else classes_of<KIND_ROUND, 64>(vals, cls);
  }
  if (vals.size() > 4) return fail(ADCT_E_ARG, "internal: more than four row classes");
  memset(&out.t, 0, sizeof(out.t));
  for (int v = 0; v < n; ++v) out.t.cls[v] = static_cast<uint8_t>(cls[v]);
  for (size_t a = 0; a < vals.size(); ++a)
    for (size_t b = 0; b < vals.size(); ++b) {
      const double dd = static_cast<double>(vals[a]) * static_cast<double>(vals[b]);
      out.t.s2[a * 4 + b] = static_cast<float>(1.0 / sqrt(dd));
      if (qstep > 0) {
        const double g = qstep * sqrt(dd);
        out.t.mq[a * 4 + b] = static_cast<int32_t>(round_half_away(16777216.0 / g));
        out.t.dq[a * 4 + b] = static_cast<int32_t>(round_half_away(2.0 * g));
      }
    }
  out.mq_full.assign(n * n, 0);
  out.dq_full.assign(n * n, 0);
  for (int v = 0; v < n; ++v)
    for (int u = 0; u < n; ++u) {
      const int ti = out.t.cls[v] * 4 + out.t.cls[u];
      out.mq_full[v * n + u] = out.t.mq[ti];
      out.dq_full[v * n + u] = out.t.dq[ti];
    }
  return ADCT_OK;
}

int pixel_bytes(int dtype) { return dtype == ADCT_U8 ? 1 : 2; }

// Common checks of a pixel image set; fills g.
int check_images(const char* what, int n, int dtype, const void* ptr, int batch, int height,
                 int width, int64_t pitch, int64_t image_stride, Geom& g) {
  if (dtype != ADCT_U8 && dtype != ADCT_I16) return fail(ADCT_E_ARG, "%s: bad dtype %d", what, dtype);
  if (n == 64 && dtype != ADCT_U8)
    return fail(ADCT_E_ARG, "%s: the 64-point transform takes 8-bit images only", what);
  if (batch < 0 || height < 0 || width < 0)
    return fail(ADCT_E_SHAPE, "%s: negative size", what);
  if (height % n || width % n)
    return fail(ADCT_E_SHAPE, "%s: %dx%d is not a multiple of n=%d", what, height, width, n);
  if (pitch < width) return fail(ADCT_E_SHAPE, "%s: pitch %lld < width %d", what, (long long)pitch, width);
  if (batch > 1 && image_stride < pitch * height)
    return fail(ADCT_E_SHAPE, "%s: image_stride %lld < pitch*height", what, (long long)image_stride);
  const int64_t align = std::min<int64_t>(16, static_cast<int64_t>(n) * pixel_bytes(dtype));
  const int64_t bytes_pitch = pitch * pixel_bytes(dtype);
  const int64_t bytes_stride = batch > 1 ? image_stride * pixel_bytes(dtype) : 0;
  if (ptr != nullptr && ((reinterpret_cast<uintptr_t>(ptr) % align) || (bytes_pitch % align) ||
                         (bytes_stride % align)))
    return fail(ADCT_E_ALIGN, "%s: images and rows must be %lld-byte aligned", what, (long long)align);
  g.pitch = pitch;
  g.image_stride = image_stride;
  g.batch = batch;
  g.tiles_y = height / n;
  g.tiles_x = width / n;
  return ADCT_OK;
}

int check_common(int transform, int n) {
  if (!valid_kind(transform)) return fail(ADCT_E_ARG, "bad transform id %d", transform);
  if (!valid_n(n)) return fail(ADCT_E_ARG, "bad block length %d (8, 16, 32 or 64)", n);
  if (!valid_kind_n(transform, n))
    return fail(ADCT_E_ARG, "transform %d is an 8-point transform (n=%d)", transform, n);
  return ADCT_OK;
}

int check_r_q(int n, int r, int qstep) {
  if (r < 1 || r > n * n) return fail(ADCT_E_ARG, "r=%d outside [1, %d]", r, n * n);
  if (qstep < 0 || qstep > 4096) return fail(ADCT_E_ARG, "qstep=%d outside [0, 4096]", qstep);
  if (n == 64 && qstep != 0) return fail(ADCT_E_ARG, "the 64-point transform is zonal only");
  return ADCT_OK;
}

int launch(Mode mode, int kind, int n, int dtype, const PassParams& p, adct_stream_t stream) {
  if (p.g.batch == 0 || p.g.tiles_x == 0 || p.g.tiles_y == 0) return ok();
  // the fused kernels decode their workgroup index in 32 bits
  const int64_t per = n == 8 ? 64 : 256 / n;
  if ((p.g.tiles_x + per - 1) / per * static_cast<int64_t>(p.g.tiles_y) * p.g.batch >=
      (int64_t(1) << 32))
    return fail(ADCT_E_SHAPE, "image set too large for one launch (2^32 workgroups)");
  const hipStream_t s = static_cast<hipStream_t>(stream);
  const int e = kind == ADCT_DCT ? launch_dct8(dtype, p, s)
                : n == 8         ? launch_n8(mode, kind, dtype, p, s)
                                 : launch_jam(mode, kind, n, dtype, p, s);
  if (e != hipSuccess)
    return fail(ADCT_E_HIP, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

// Scratch of adct_compress_quality_noalloc: the error energies and moment
// records of one call, in a fixed array of device memory that every GPU the
// library runs on holds until the process ends (4 MiB).  Host code uses the
// per-device address from hipGetSymbolAddress, never the array's name.
constexpr int64_t kScratchWords = int64_t(1) << 19;
static __device__ __align__(256) unsigned long long scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned long long* g_scratch_ptr[kMaxDevices] = {};

// The scratch array's address on the current device, looked up once per
// device (with that device current).
int static_scratch(unsigned long long** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(ADCT_E_HIP, "hipGetDevice failed: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(ADCT_E_HIP, "device %d out of range", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || ptr == nullptr)
      return fail(ADCT_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<unsigned long long*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return ADCT_OK;
}

// Words of the compress-with-quality workspace: one error energy per image,
// then one moment record per image when the coding gain is wanted.
int64_t quality_words(int n, int batch, bool with_cg) {
  return static_cast<int64_t>(batch) * (1 + (with_cg ? 3 * n * n + 4 : 0));
}

// adct_compress followed by PSNR and (optionally) the measured coding gain;
// the error energies and moment records live in `work` (`words` 64-bit
// words), zeroed here with a fill kernel.
int static_scratch(unsigned long long** out);

int compress_quality(const char* what, int transform, int n, int r, int qstep, const void* d_src,
                     int dtype, int batch, int height, int width, int64_t pitch,
                     int64_t image_stride, int32_t* d_kept, float* d_scaled, void* d_recon,
                     float* d_psnr, float* d_cg, int basis, unsigned long long* work,
                     int64_t words, bool use_static_scratch, adct_stream_t stream) {
  if (int s = check_common(transform, n)) return s;
  if (int s = check_r_q(n, r, qstep)) return s;
  if (basis != ADCT_BASIS_ROWS && basis != ADCT_BASIS_COLS)
    return fail(ADCT_E_ARG, "%s: bad basis %d", what, basis);
  PassParams p{};
  if (int s = check_images(what, n, dtype, d_src, batch, height, width, pitch, image_stride, p.g))
    return s;
  if (p.g.batch == 0 || p.g.tiles_x == 0 || p.g.tiles_y == 0) return ok();
  if (d_src == nullptr) return fail(ADCT_E_ARG, "%s: null source", what);
  if (d_recon != nullptr && (reinterpret_cast<uintptr_t>(d_recon) %
                             std::min<int64_t>(16, static_cast<int64_t>(n) * pixel_bytes(dtype))))
    return fail(ADCT_E_ALIGN, "%s: misaligned reconstruction buffer", what);
  if ((reinterpret_cast<uintptr_t>(d_kept) % 4) || (reinterpret_cast<uintptr_t>(d_scaled) % 4) ||
      (reinterpret_cast<uintptr_t>(d_psnr) % 4) || (reinterpret_cast<uintptr_t>(d_cg) % 4))
    return fail(ADCT_E_ALIGN, "%s: misaligned output buffer", what);
  const int64_t need = quality_words(n, batch, d_cg != nullptr);
  if (words < need)
    return fail(ADCT_E_BUDGET, "%s: the workspace holds %lld words, %lld needed", what,
                (long long)words, (long long)need);
  if (static_cast<int64_t>(p.g.tiles_x) * p.g.tiles_y >= (int64_t(1) << 32))
    return fail(ADCT_E_SHAPE, "%s: more than 2^32 tiles per image", what);
  if (transform == ADCT_DCT && (qstep != 0 || d_kept != nullptr || d_cg != nullptr))
    return fail(ADCT_E_ARG, "%s: the DCT path is zonal, without integer coefficients or "
                            "moments", what);
  TableSet ts;
  if (transform != ADCT_DCT)
    if (int s = build_tables(transform, n, qstep, ts)) return s;
  if (use_static_scratch)
    if (int s = static_scratch(&work)) return s;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  int e = launch_fill_zero(work, need, st);
  if (e != hipSuccess)
    return fail(ADCT_E_HIP, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  p.t = ts.t;
  p.src = d_src;
  p.dst = d_recon;
  p.cout = d_kept;
  p.scaled = d_scaled;
  p.sse = work;
  p.r = r;
  p.qstep = qstep;
  if (int s = launch(Mode::Compress, transform, n, dtype, p, stream)) return s;
  const int64_t pixels = static_cast<int64_t>(height) * width;
  if (d_psnr != nullptr) e = launch_psnr(work, batch, pixels, d_psnr, st);
  if (e == hipSuccess && d_cg != nullptr) {
    e = launch_moments(transform, n, dtype, d_src, p.g, work + batch, st);
    if (e == hipSuccess) e = launch_coding_gain(transform, n, basis, work + batch, batch, d_cg, st);
  }
  if (e != hipSuccess)
    return fail(ADCT_E_HIP, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

}  // namespace

int set_error(int status, const char* msg) {
  if (status == ADCT_OK) g_last_error.clear();
  else g_last_error = msg;
  return status;
}

int build_tables_for(int kind, int n, int qstep, Tables* out) {
  TableSet ts;
  if (int s = build_tables(kind, n, qstep, ts)) return s;
  *out = ts.t;
  return ADCT_OK;
}

}  // namespace adct

using namespace adct;

extern "C" {

ADCT_API int adct_version(void) { return 1; }

ADCT_API const char* adct_last_error(void) { return g_last_error.c_str(); }

ADCT_API int adct_get_matrix(int transform, int n, int inverse, int32_t* host_out) {
  if (int s = check_common(transform, n)) return s;
  if (transform == ADCT_DCT) return fail(ADCT_E_ARG, "get_matrix: the DCT is not an integer matrix");
  if (host_out == nullptr) return fail(ADCT_E_ARG, "null output");
  std::vector<int> m;
  operator_matrix(transform, n, inverse != 0, m);
  for (int i = 0; i < n * n; ++i) {
    if (inverse) {
      // the inverse butterfly applies K_N = 2 U_N
      if (m[i] % 2) return fail(ADCT_E_ARG, "internal: odd entry in the inverse chain");
      host_out[i] = m[i] / 2;
    } else {
      host_out[i] = m[i];
    }
  }
  return ok();
}

ADCT_API int adct_transform_measures(int transform, int n, double* eps, double* delta) {
  if (int s = check_common(transform, n)) return s;
  if (eps == nullptr && delta == nullptr) return fail(ADCT_E_ARG, "null output");
  if (transform == ADCT_DCT) {   // the reference itself
    if (eps) *eps = 0.0;
    if (delta) *delta = 0.0;
    return ok();
  }
  std::vector<int> t;
  operator_matrix(transform, n, false, t);
  std::vector<double> s(n);
  for (int v = 0; v < n; ++v) {
    double d = 0.0;
    for (int i = 0; i < n; ++i) d += static_cast<double>(t[v * n + i]) * t[v * n + i];
    s[v] = 1.0 / sqrt(d);
  }
  if (eps != nullptr) {
    // pi ||C - S T||_F^2 with C the orthonormal DCT-II (section 4.1, Table 1)
    double e = 0.0;
    for (int v = 0; v < n; ++v)
      for (int i = 0; i < n; ++i) {
        const double c = sqrt(2.0 / n) * (v == 0 ? sqrt(0.5) : 1.0) *
                         cos(v * (2 * i + 1) * M_PI / (2.0 * n));
        const double dlt = c - s[v] * t[v * n + i];
        e += dlt * dlt;
      }
    *eps = M_PI * e;
  }
  if (delta != nullptr) {
    // 1 - ||diag(M)||^2 / ||M||_F^2 for M = T T^T (section 3.1)
    double dg = 0.0, all = 0.0;
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) {
        double m = 0.0;
        for (int i = 0; i < n; ++i) m += static_cast<double>(t[a * n + i]) * t[b * n + i];
        all += m * m;
        if (a == b) dg += m * m;
      }
    *delta = 1.0 - dg / all;
  }
  return ok();
}

ADCT_API int adct_zigzag(int n, int32_t* host_out) {
  if (!valid_n(n)) return fail(ADCT_E_ARG, "bad block length %d", n);
  if (host_out == nullptr) return fail(ADCT_E_ARG, "null output");
  for (int v = 0; v < n; ++v)
    for (int u = 0; u < n; ++u) host_out[zz_pos(n, v, u)] = v * n + u;
  return ok();
}

ADCT_API int adct_scale_vector(int transform, int n, double* host_out) {
  if (int s = check_common(transform, n)) return s;
  if (host_out == nullptr) return fail(ADCT_E_ARG, "null output");
  if (transform == ADCT_DCT) {   // already orthonormal
    for (int i = 0; i < n; ++i) host_out[i] = 1.0;
    return ok();
  }
  std::vector<int64_t> d;
  diag_ttt(transform, n, d);
  for (int i = 0; i < n; ++i) host_out[i] = 1.0 / sqrt(static_cast<double>(d[i]));
  return ok();
}

ADCT_API int adct_quant_tables(int transform, int n, int qstep, int32_t* mq, int32_t* dq) {
  if (int s = check_common(transform, n)) return s;
  if (transform == ADCT_DCT) return fail(ADCT_E_ARG, "quant_tables: the DCT path is zonal only");
  if (qstep < 1 || qstep > 4096) return fail(ADCT_E_ARG, "qstep=%d outside [1, 4096]", qstep);
  TableSet ts;
  if (int s = build_tables(transform, n, qstep, ts)) return s;
  for (int i = 0; i < n * n; ++i) {
    if (mq) mq[i] = ts.mq_full[i];
    if (dq) dq[i] = ts.dq_full[i];
  }
  return ok();
}

ADCT_API int adct_fwd2d(int transform, int n, const void* d_src, int dtype, int batch, int height,
                        int width, int64_t pitch, int64_t image_stride, int32_t* d_coef,
                        adct_stream_t stream) {
  if (int s = check_common(transform, n)) return s;
  if (transform == ADCT_DCT) return fail(ADCT_E_ARG, "fwd2d: the DCT has no integer coefficients");
  PassParams p{};
  if (int s = check_images("fwd2d", n, dtype, d_src, batch, height, width, pitch, image_stride, p.g))
    return s;
  if (p.g.batch == 0 || p.g.tiles_x == 0 || p.g.tiles_y == 0) return ok();
  if (d_src == nullptr || d_coef == nullptr) return fail(ADCT_E_ARG, "fwd2d: null pointer");
  if (reinterpret_cast<uintptr_t>(d_coef) % 16) return fail(ADCT_E_ALIGN, "fwd2d: d_coef must be 16-byte aligned");
  p.src = d_src;
  p.cout = d_coef;
  p.r = n * n;
  return launch(Mode::Forward, transform, n, dtype, p, stream);
}

static int inverse_common(Mode mode, int transform, int n, int r, int qstep, const int32_t* d_in,
                          void* d_dst, int dtype, int batch, int height, int width, int64_t pitch,
                          int64_t image_stride, adct_stream_t stream) {
  if (int s = check_common(transform, n)) return s;
  if (transform == ADCT_DCT) return fail(ADCT_E_ARG, "inverse: the DCT has no integer coefficients");
  if (int s = check_r_q(n, r, qstep)) return s;
  PassParams p{};
  if (int s = check_images("inverse", n, dtype, d_dst, batch, height, width, pitch, image_stride, p.g))
    return s;
  if (p.g.batch == 0 || p.g.tiles_x == 0 || p.g.tiles_y == 0) return ok();
  if (d_in == nullptr || d_dst == nullptr) return fail(ADCT_E_ARG, "inverse: null pointer");
  if (mode == Mode::Inverse && reinterpret_cast<uintptr_t>(d_in) % 16)
    return fail(ADCT_E_ALIGN, "inv2d: d_coef must be 16-byte aligned");
  if (reinterpret_cast<uintptr_t>(d_in) % 4) return fail(ADCT_E_ALIGN, "inverse: misaligned input");
  TableSet ts;
  if (int s = build_tables(transform, n, qstep, ts)) return s;
  p.t = ts.t;
  p.cin = d_in;
  p.dst = d_dst;
  p.r = r;
  p.qstep = qstep;
  return launch(mode, transform, n, dtype, p, stream);
}

ADCT_API int adct_inv2d(int transform, int n, int r, int qstep, const int32_t* d_coef, void* d_dst,
                        int dtype, int batch, int height, int width, int64_t pitch,
                        int64_t image_stride, adct_stream_t stream) {
  return inverse_common(Mode::Inverse, transform, n, r, qstep, d_coef, d_dst, dtype, batch, height,
                        width, pitch, image_stride, stream);
}

ADCT_API int adct_decompress(int transform, int n, int r, int qstep, const int32_t* d_kept,
                             void* d_dst, int dtype, int batch, int height, int width,
                             int64_t pitch, int64_t image_stride, adct_stream_t stream) {
  return inverse_common(Mode::Decompress, transform, n, r, qstep, d_kept, d_dst, dtype, batch,
                        height, width, pitch, image_stride, stream);
}

ADCT_API int adct_compress(int transform, int n, int r, int qstep, const void* d_src, int dtype,
                           int batch, int height, int width, int64_t pitch, int64_t image_stride,
                           int32_t* d_kept, float* d_scaled, void* d_recon, uint64_t* d_sse,
                           adct_stream_t stream) {
  if (int s = check_common(transform, n)) return s;
  if (int s = check_r_q(n, r, qstep)) return s;
  PassParams p{};
  if (int s = check_images("compress", n, dtype, d_src, batch, height, width, pitch, image_stride, p.g))
    return s;
  if (p.g.batch == 0 || p.g.tiles_x == 0 || p.g.tiles_y == 0) return ok();
  if (d_src == nullptr) return fail(ADCT_E_ARG, "compress: null source");
  if (d_recon != nullptr && (reinterpret_cast<uintptr_t>(d_recon) %
                             std::min<int64_t>(16, static_cast<int64_t>(n) * pixel_bytes(dtype))))
    return fail(ADCT_E_ALIGN, "compress: misaligned reconstruction buffer");
  if ((reinterpret_cast<uintptr_t>(d_kept) % 4) || (reinterpret_cast<uintptr_t>(d_scaled) % 4) ||
      (reinterpret_cast<uintptr_t>(d_sse) % 8))
    return fail(ADCT_E_ALIGN, "compress: misaligned output buffer");
  if (transform == ADCT_DCT && (qstep != 0 || d_kept != nullptr))
    return fail(ADCT_E_ARG, "compress: the DCT path is zonal and has no integer coefficients "
                            "(qstep 0, d_kept NULL; d_scaled receives its coefficients)");
  TableSet ts;
  if (transform != ADCT_DCT)
    if (int s = build_tables(transform, n, qstep, ts)) return s;
  p.t = ts.t;
  p.src = d_src;
  p.dst = d_recon;
  p.cout = d_kept;
  p.scaled = d_scaled;
  p.sse = reinterpret_cast<unsigned long long*>(d_sse);
  p.r = r;
  p.qstep = qstep;
  return launch(Mode::Compress, transform, n, dtype, p, stream);
}

ADCT_API int adct_compress_mfma(int transform, int r, const void* d_src, int batch, int height,
                                int width, int64_t pitch, int64_t image_stride, int32_t* d_kept,
                                float* d_scaled, void* d_recon, uint64_t* d_sse,
                                adct_stream_t stream) {
  const int n = 8;
  if (int s = check_common(transform, n)) return s;
  if (transform == ADCT_DCT) return fail(ADCT_E_ARG, "compress_mfma: integer transforms only");
  if (int s = check_r_q(n, r, 0)) return s;
  PassParams p{};
  if (int s = check_images("compress_mfma", n, ADCT_U8, d_src, batch, height, width, pitch,
                           image_stride, p.g))
    return s;
  if (p.g.batch == 0 || p.g.tiles_x == 0 || p.g.tiles_y == 0) return ok();
  if (d_src == nullptr) return fail(ADCT_E_ARG, "compress_mfma: null source");
  if ((reinterpret_cast<uintptr_t>(d_recon) % 8) || (reinterpret_cast<uintptr_t>(d_kept) % 4) ||
      (reinterpret_cast<uintptr_t>(d_scaled) % 4) || (reinterpret_cast<uintptr_t>(d_sse) % 8))
    return fail(ADCT_E_ALIGN, "compress_mfma: misaligned output buffer");
  TableSet ts;
  if (int s = build_tables(transform, n, 0, ts)) return s;
  p.t = ts.t;
  p.src = d_src;
  p.dst = d_recon;
  p.cout = d_kept;
  p.scaled = d_scaled;
  p.sse = reinterpret_cast<unsigned long long*>(d_sse);
  p.r = r;
  std::vector<int> fwd, inv;
  operator_matrix(transform, n, false, fwd);
  operator_matrix(transform, n, true, inv);
  int8_t t8m[64], u8m[64];
  for (int i = 0; i < 64; ++i) {
    // the inverse butterfly applies 2 U; U = 8 T^-1 has entries in {0, +-1, +-2}
    if (fwd[i] < -2 || fwd[i] > 2 || inv[i] % 2 || inv[i] < -4 || inv[i] > 4)
      return fail(ADCT_E_ARG, "internal: matrix entry outside the int8 operand range");
    t8m[i] = static_cast<int8_t>(fwd[i]);
    u8m[i] = static_cast<int8_t>(inv[i] / 2);
  }
  const int e = launch_n8_mfma(transform, p, t8m, u8m, static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return fail(ADCT_E_HIP, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

ADCT_API int64_t adct_compress_quality_workspace(int n, int batch, int with_coding_gain) {
  if (!valid_n(n) || batch < 0) return fail(ADCT_E_ARG, "quality workspace: bad n or batch");
  return 8 * quality_words(n, batch, with_coding_gain != 0);
}

ADCT_API int adct_compress_quality(int transform, int n, int r, int qstep, const void* d_src,
                                   int dtype, int batch, int height, int width, int64_t pitch,
                                   int64_t image_stride, int32_t* d_kept, float* d_scaled,
                                   void* d_recon, float* d_psnr, float* d_cg, int basis,
                                   void* d_work, int64_t work_bytes, adct_stream_t stream) {
  if (d_work == nullptr && batch > 0) return fail(ADCT_E_ARG, "compress_quality: null workspace");
  if (reinterpret_cast<uintptr_t>(d_work) % 8)
    return fail(ADCT_E_ALIGN, "compress_quality: misaligned workspace");
  return compress_quality("compress_quality", transform, n, r, qstep, d_src, dtype, batch, height,
                          width, pitch, image_stride, d_kept, d_scaled, d_recon, d_psnr, d_cg,
                          basis, static_cast<unsigned long long*>(d_work),
                          work_bytes < 0 ? 0 : work_bytes / 8, false, stream);
}

ADCT_API int adct_compress_quality_noalloc(int transform, int n, int r, int qstep,
                                           const void* d_src, int dtype, int batch, int height,
                                           int width, int64_t pitch, int64_t image_stride,
                                           int32_t* d_kept, float* d_scaled, void* d_recon,
                                           float* d_psnr, float* d_cg, int basis,
                                           adct_stream_t stream) {
  return compress_quality("compress_quality_noalloc", transform, n, r, qstep, d_src, dtype, batch,
                          height, width, pitch, image_stride, d_kept, d_scaled, d_recon, d_psnr,
                          d_cg, basis, nullptr, kScratchWords, true, stream);
}

ADCT_API int adct_ssim(const void* d_x, const void* d_y, int batch, int height, int width,
                       int64_t pitch, int64_t image_stride, double* d_work, float* d_ssim,
                       adct_stream_t stream) {
  if (batch < 0 || height < 0 || width < 0) return fail(ADCT_E_SHAPE, "ssim: negative size");
  if (batch == 0) return ok();
  if (height < 11 || width < 11)
    return fail(ADCT_E_SHAPE, "ssim: %dx%d is smaller than the 11x11 window", height, width);
  if (pitch < width) return fail(ADCT_E_SHAPE, "ssim: pitch %lld < width %d", (long long)pitch, width);
  if (batch > 1 && image_stride < pitch * height)
    return fail(ADCT_E_SHAPE, "ssim: image_stride %lld < pitch*height", (long long)image_stride);
  if (d_x == nullptr || d_y == nullptr || d_work == nullptr || d_ssim == nullptr)
    return fail(ADCT_E_ARG, "ssim: null pointer");
  if ((reinterpret_cast<uintptr_t>(d_work) % 8) || (reinterpret_cast<uintptr_t>(d_ssim) % 4))
    return fail(ADCT_E_ALIGN, "ssim: misaligned buffer");
  const int e = launch_ssim(static_cast<const uint8_t*>(d_x), static_cast<const uint8_t*>(d_y),
                            batch, height, width, pitch, image_stride, d_work, d_ssim,
                            static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return fail(ADCT_E_HIP, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

ADCT_API int adct_ape(int count, const float* d_value, const float* d_reference, float* d_ape,
                      adct_stream_t stream) {
  if (count < 0) return fail(ADCT_E_ARG, "ape: negative count");
  if (count == 0) return ok();
  if (d_value == nullptr || d_reference == nullptr || d_ape == nullptr)
    return fail(ADCT_E_ARG, "ape: null pointer");
  if ((reinterpret_cast<uintptr_t>(d_value) % 4) || (reinterpret_cast<uintptr_t>(d_reference) % 4) ||
      (reinterpret_cast<uintptr_t>(d_ape) % 4))
    return fail(ADCT_E_ALIGN, "ape: misaligned buffer");
  const int e = launch_ape(d_value, d_reference, count, d_ape, static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return fail(ADCT_E_HIP, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

ADCT_API int adct_psnr(int count, int64_t pixels, const uint64_t* d_sse, float* d_psnr,
                       adct_stream_t stream) {
  if (count < 0) return fail(ADCT_E_ARG, "psnr: negative count");
  if (count == 0) return ok();
  if (pixels < 1) return fail(ADCT_E_ARG, "psnr: pixels must be positive");
  if (d_sse == nullptr || d_psnr == nullptr) return fail(ADCT_E_ARG, "psnr: null pointer");
  if ((reinterpret_cast<uintptr_t>(d_sse) % 8) || (reinterpret_cast<uintptr_t>(d_psnr) % 4))
    return fail(ADCT_E_ALIGN, "psnr: misaligned buffer");
  const int e = launch_psnr(reinterpret_cast<const unsigned long long*>(d_sse), count, pixels,
                            d_psnr, static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return fail(ADCT_E_HIP, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

ADCT_API int adct_moments(int transform, int n, const void* d_src, int dtype, int batch,
                          int height, int width, int64_t pitch, int64_t image_stride,
                          uint64_t* d_moments, adct_stream_t stream) {
  if (int s = check_common(transform, n)) return s;
  if (transform == ADCT_DCT) return fail(ADCT_E_ARG, "moments: integer transforms only");
  Geom g{};
  if (int s = check_images("moments", n, dtype, d_src, batch, height, width, pitch, image_stride, g))
    return s;
  if (g.batch == 0 || g.tiles_x == 0 || g.tiles_y == 0) return ok();
  if (d_src == nullptr || d_moments == nullptr) return fail(ADCT_E_ARG, "moments: null pointer");
  if (reinterpret_cast<uintptr_t>(d_moments) % 8) return fail(ADCT_E_ALIGN, "moments: misaligned records");
  if (static_cast<int64_t>(g.tiles_x) * g.tiles_y >= (int64_t(1) << 32))
    return fail(ADCT_E_SHAPE, "moments: more than 2^32 tiles per image");
  const int e = launch_moments(transform, n, dtype, d_src, g,
                               reinterpret_cast<unsigned long long*>(d_moments),
                               static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return fail(ADCT_E_HIP, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

ADCT_API int adct_coding_gain(int transform, int n, int basis, int count,
                              const uint64_t* d_moments, float* d_cg, adct_stream_t stream) {
  if (int s = check_common(transform, n)) return s;
  if (transform == ADCT_DCT) return fail(ADCT_E_ARG, "coding_gain: integer transforms only");
  if (basis != ADCT_BASIS_ROWS && basis != ADCT_BASIS_COLS)
    return fail(ADCT_E_ARG, "coding_gain: bad basis %d", basis);
  if (count < 0) return fail(ADCT_E_ARG, "coding_gain: negative count");
  if (count == 0) return ok();
  if (d_moments == nullptr || d_cg == nullptr) return fail(ADCT_E_ARG, "coding_gain: null pointer");
  if ((reinterpret_cast<uintptr_t>(d_moments) % 8) || (reinterpret_cast<uintptr_t>(d_cg) % 4))
    return fail(ADCT_E_ALIGN, "coding_gain: misaligned buffer");
  const int e = launch_coding_gain(transform, n, basis,
                                   reinterpret_cast<const unsigned long long*>(d_moments), count,
                                   d_cg, static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return fail(ADCT_E_HIP, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

ADCT_API int adct_coding_gain_ar1(int transform, int n, int basis, int count,
                                  const float* d_rho, float* d_cg, float* d_cg_klt,
                                  adct_stream_t stream) {
  if (int s = check_common(transform, n)) return s;
  if (transform == ADCT_DCT) return fail(ADCT_E_ARG, "coding_gain_ar1: integer transforms only");
  if (basis != ADCT_BASIS_ROWS && basis != ADCT_BASIS_COLS)
    return fail(ADCT_E_ARG, "coding_gain_ar1: bad basis %d", basis);
  if (count < 0) return fail(ADCT_E_ARG, "coding_gain_ar1: negative count");
  if (count == 0 || (d_cg == nullptr && d_cg_klt == nullptr)) return ok();
  if (d_rho == nullptr) return fail(ADCT_E_ARG, "coding_gain_ar1: null rho");
  if ((reinterpret_cast<uintptr_t>(d_rho) % 4) || (reinterpret_cast<uintptr_t>(d_cg) % 4) ||
      (reinterpret_cast<uintptr_t>(d_cg_klt) % 4))
    return fail(ADCT_E_ALIGN, "coding_gain_ar1: misaligned buffer");
  const int e = launch_coding_gain_ar1(transform, n, basis, d_rho, count, d_cg, d_cg_klt,
                                       static_cast<hipStream_t>(stream));
  if (e != hipSuccess)
    return fail(ADCT_E_HIP, "kernel launch failed: %s", hipGetErrorString(static_cast<hipError_t>(e)));
  return ok();
}

}  // extern "C"
