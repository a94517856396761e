// Structural similarity (SSIM) of an 8-bit image and its reconstruction, the
// second quality measure of section 5.1 (the paper cites the index of Wang,
// Bovik, Sheikh and Simoncelli): for every full 11 x 11 window,
//   SSIM = (2 mu_x mu_y + C1)(2 s_xy + C2) / ((mu_x^2 + mu_y^2 + C1)(s_x^2 + s_y^2 + C2))
// with means, variances and the covariance weighted by a normalised Gaussian
// (sigma 1.5), C1 = (0.01 * 255)^2, C2 = (0.03 * 255)^2; the image's SSIM is
// the mean over its (H - 10) x (W - 10) windows.
//
// A 256-thread workgroup owns 16 x 64 windows.  It stages the 26 x 74 pixels
// of both images those windows cover in LDS (as floats, shifted by the
// region's top-left pixel so that the window moments are formed from small
// numbers: variances and the covariance do not change under a shift, and the
// means get it back), runs the separable Gaussian along rows for the five
// moments (x, y, x^2, y^2, x y), then along columns, evaluates the index of
// each window in float32, sums the workgroup's windows by a fixed-order tree
// and adds the sum to the image's float64 accumulator.  A last kernel
// divides by the window count.
#include <algorithm>

#include "adct_internal.hpp"

namespace adct {
namespace {

constexpr int kOW = 64;            // windows per workgroup, horizontally
constexpr int kOH = 16;            // and vertically
constexpr int kK = 11;             // window size
constexpr int kRW = kOW + kK - 1;  // 74 pixels of a region row
constexpr int kRH = kOH + kK - 1;  // 26 region rows
constexpr int kBS = 256;

// Normalised 11-tap Gaussian, sigma 1.5 (the 2D window is its outer product).
struct Gauss {
  float g[kK];
};

constexpr double cexp(double x) {   // exp for the compile-time table (|x| < 12)
  double term = 1.0, sum = 1.0;
  for (int k = 1; k < 80; ++k) {
    term *= x / k;
    sum += term;
  }
  return sum;
}

constexpr Gauss make_gauss() {
  double w[kK] = {};
  double s = 0.0;
  for (int i = 0; i < kK; ++i) {
    const double t = i - kK / 2;
    w[i] = 1.0 / cexp(t * t / (2.0 * 1.5 * 1.5));
    s += w[i];
  }
  Gauss g{};
  for (int i = 0; i < kK; ++i) g.g[i] = static_cast<float>(w[i] / s);
  return g;
}

static __constant__ Gauss kGauss = make_gauss();

struct SsimParams {
  const uint8_t* x;
  const uint8_t* y;
  int64_t pitch, image_stride;
  int height, width;
  double* acc;   // [batch] sums of the windows' index
};

__global__ __launch_bounds__(kBS) void ssim_kernel(SsimParams p) {
  __shared__ float X[kRH][kRW], Y[kRH][kRW];
  __shared__ float Hs[5][kRH][kOW];
  __shared__ float red[kBS / 64];
  const int img = blockIdx.z;
  const int wx0 = blockIdx.x * kOW, wy0 = blockIdx.y * kOH;   // first window (its top-left pixel)
  const int nwx = p.width - kK + 1, nwy = p.height - kK + 1;  // windows per row / column
  const int64_t base = img * p.image_stride;
  const uint8_t* xs = p.x + base;
  const uint8_t* ys = p.y + base;
  const float sx = static_cast<float>(xs[static_cast<int64_t>(wy0) * p.pitch + wx0]);
  const float sy = static_cast<float>(ys[static_cast<int64_t>(wy0) * p.pitch + wx0]);
  for (int e = threadIdx.x; e < kRH * kRW; e += kBS) {
    const int r = e / kRW, c = e - r * kRW;
    const int yy = wy0 + r, xx = wx0 + c;
    float vx = 0.0f, vy = 0.0f;
    if (yy < p.height && xx < p.width) {
      const int64_t o = static_cast<int64_t>(yy) * p.pitch + xx;
      vx = static_cast<float>(xs[o]) - sx;
      vy = static_cast<float>(ys[o]) - sy;
    }
    X[r][c] = vx;
    Y[r][c] = vy;
  }
  __syncthreads();
  // rows: the five moments of every region row at every window column
  for (int e = threadIdx.x; e < kRH * kOW; e += kBS) {
    const int r = e / kOW, c = e - r * kOW;
    float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int j = 0; j < kK; ++j) {
      const float g = kGauss.g[j], a = X[r][c + j], b = Y[r][c + j];
      m[0] = fmaf(g, a, m[0]);
      m[1] = fmaf(g, b, m[1]);
      m[2] = fmaf(g, a * a, m[2]);
      m[3] = fmaf(g, b * b, m[3]);
      m[4] = fmaf(g, a * b, m[4]);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) Hs[q][r][c] = m[q];
  }
  __syncthreads();
  // columns, then the index of every window of the workgroup
  constexpr float C1 = (0.01f * 255.0f) * (0.01f * 255.0f);
  constexpr float C2 = (0.03f * 255.0f) * (0.03f * 255.0f);
  float sum = 0.0f;
  for (int e = threadIdx.x; e < kOH * kOW; e += kBS) {
    const int r = e / kOW, c = e - r * kOW;
    if (wy0 + r >= nwy || wx0 + c >= nwx) continue;
    float m[5] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int i = 0; i < kK; ++i) {
      const float g = kGauss.g[i];
#pragma unroll
      for (int q = 0; q < 5; ++q) m[q] = fmaf(g, Hs[q][r + i][c], m[q]);
    }
    const float vx = m[2] - m[0] * m[0], vy = m[3] - m[1] * m[1], cxy = m[4] - m[0] * m[1];
    const float mx = m[0] + sx, my = m[1] + sy;
    const float num = (2.0f * mx * my + C1) * (2.0f * cxy + C2);
    const float den = (mx * mx + my * my + C1) * (vx + vy + C2);
    sum += num / den;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_xor(sum, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sum;
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.0f;
#pragma unroll
    for (int w = 0; w < kBS / 64; ++w) s += red[w];
    atomicAdd(p.acc + img, static_cast<double>(s));
  }
}

__global__ void ssim_mean_kernel(const double* acc, int count, double windows, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = static_cast<float>(acc[i] / windows);
}

__global__ void ape_kernel(const float* value, const float* ref, int count, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = 100.0f * fabsf(value[i] - ref[i]) / fabsf(ref[i]);
}

}  // namespace

int launch_ssim(const uint8_t* x, const uint8_t* y, int batch, int height, int width,
                int64_t pitch, int64_t image_stride, double* acc, float* out, hipStream_t s) {
  int e = launch_fill_zero(reinterpret_cast<unsigned long long*>(acc), batch, s);
  if (e != hipSuccess) return e;
  SsimParams p{x, y, pitch, image_stride, height, width, acc};
  const int nwx = width - kK + 1, nwy = height - kK + 1;
  const dim3 grid((nwx + kOW - 1) / kOW, (nwy + kOH - 1) / kOH, batch);
  ssim_kernel<<<grid, kBS, 0, s>>>(p);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  ssim_mean_kernel<<<(batch + 255) / 256, 256, 0, s>>>(
      acc, batch, static_cast<double>(nwx) * static_cast<double>(nwy), out);
  return hipGetLastError();
}

int launch_ape(const float* value, const float* ref, int count, float* out, hipStream_t s) {
  ape_kernel<<<(count + 255) / 256, 256, 0, s>>>(value, ref, count, out);
  return hipGetLastError();
}

}  // namespace adct
