// Quality measures of the block transform (sections 4.1 and 5.1):
//
//   moments     per image, over its tiles, the sum and the sum of squares of
//               every coefficient b[v][u] of B = T A T^T, and the sum and sum
//               of squares of the (level-shifted) pixels.  These are exact
//               integers; the measured coding gain follows from them.
//   coding gain (measured) the unified coding gain of the separable 2D
//               transform with the model's covariances replaced by the
//               variances measured over an image's tiles, in float32.
//   coding gain (AR(1)) the closed form of section 4.1 under the first-order
//               Markov model, and the KLT's, for many correlation values at
//               once, in float32.
//   PSNR        10 log10(255^2 H W / SSE) per image, in float32.
//
// For N >= 16 the moment kernel reuses the row-group code of the 16/32-point
// kernels: a 256-thread workgroup transforms 256/N horizontally adjacent
// tiles (row pass, LDS exchange, column pass) and stages all N^2
// coefficients of each tile in LDS.  Thread t then owns coefficient
// positions t, t + 256, ... and keeps running sums of them in registers
// while the workgroup walks its share of the image's tile groups; one set of
// 64-bit atomics per workgroup adds them to the image's record.  For N = 8
// one thread owns one tile (as in the fused 8-point kernels) and one-wave
// workgroups exchange the coefficients through LDS, lane p summing position
// p.  Squares are split into their low and high 32-bit halves, each summed
// in 64 bits, so every sum is exact for any int16 input (for 8-bit input the
// bound on |b| lets runs of squares be summed in 32 bits first).
#include <algorithm>
#include <type_traits>

#include "jam_group.hpp"
#include "tile8.hpp"

namespace adct {
namespace {

using namespace jam;

// ------------------------------------------------------- transform constants
// T_N, diag(T T^T) and the norms behind B_k, all from the butterflies at
// compile time (U = N T^-1 is half of the inverse chain K_N).
template <int N>
struct TransformInfo {
  int8_t t[N][N];        // T_N, row-major
  int32_t d[N];          // diag(T T^T)
  int32_t ucol2[N];      // sum_j U[j][k]^2: squared norm of column k of U
  int64_t urow2d[N];     // sum_j U[k][j]^2 d_j
  int32_t l1max;         // largest row sum of |T[v][i]|
};

template <int KIND, int N>
constexpr TransformInfo<N> make_info() {
  TransformInfo<N> I{};
  int u[N][N] = {};
  for (int j = 0; j < N; ++j) {
    int e[N] = {};
    e[j] = 1;
    fwdN<KIND, N>(e);
    for (int v = 0; v < N; ++v) I.t[v][j] = static_cast<int8_t>(e[v]);
    int f[N] = {};
    f[j] = 1;
    invN<KIND, N>(f);
    for (int v = 0; v < N; ++v) u[v][j] = f[v] / 2;
  }
  I.l1max = 0;
  for (int v = 0; v < N; ++v) {
    int d = 0, l1 = 0, c2 = 0;
    for (int i = 0; i < N; ++i) {
      d += I.t[v][i] * I.t[v][i];
      l1 += I.t[v][i] < 0 ? -I.t[v][i] : I.t[v][i];
      c2 += u[i][v] * u[i][v];
    }
    I.d[v] = d;
    I.ucol2[v] = c2;
    if (l1 > I.l1max) I.l1max = l1;
  }
  for (int v = 0; v < N; ++v) {
    int64_t s = 0;
    for (int i = 0; i < N; ++i) s += static_cast<int64_t>(u[v][i]) * u[v][i] * I.d[i];
    I.urow2d[v] = s;
  }
  return I;
}

static __constant__ TransformInfo<8> kInfo1_8 = make_info<KIND_SIGN, 8>();
static __constant__ TransformInfo<16> kInfo1_16 = make_info<KIND_SIGN, 16>();
static __constant__ TransformInfo<32> kInfo1_32 = make_info<KIND_SIGN, 32>();
static __constant__ TransformInfo<8> kInfo2_8 = make_info<KIND_ROUND, 8>();
static __constant__ TransformInfo<16> kInfo2_16 = make_info<KIND_ROUND, 16>();
static __constant__ TransformInfo<32> kInfo2_32 = make_info<KIND_ROUND, 32>();
static __constant__ TransformInfo<64> kInfo1_64 = make_info<KIND_SIGN, 64>();
static __constant__ TransformInfo<64> kInfo2_64 = make_info<KIND_ROUND, 64>();
static __constant__ TransformInfo<8> kInfoWHT = make_info<KIND_WHT, 8>();
static __constant__ TransformInfo<8> kInfoSDCT = make_info<KIND_SDCT, 8>();
static __constant__ TransformInfo<8> kInfoHT = make_info<KIND_HT, 8>();

template <int KIND, int N>
__device__ __forceinline__ const TransformInfo<N>& info() {
  if constexpr (KIND == KIND_WHT) {
    return kInfoWHT;
  } else if constexpr (KIND == KIND_SDCT) {
    return kInfoSDCT;
  } else if constexpr (KIND == KIND_HT) {
    return kInfoHT;
  } else if constexpr (KIND == KIND_SIGN) {
    if constexpr (N == 8) return kInfo1_8;
    else if constexpr (N == 16) return kInfo1_16;
    else if constexpr (N == 32) return kInfo1_32;
    else return kInfo1_64;
  } else {
    if constexpr (N == 8) return kInfo2_8;
    else if constexpr (N == 16) return kInfo2_16;
    else if constexpr (N == 32) return kInfo2_32;
    else return kInfo2_64;
  }
}

// B_k of section 4.1 times the 1/d_k that the scale s_k^2 contributes to A_k,
// for the columns (synthesis basis) or the rows of C^-1 = (U / N) S^-1:
//   columns: B_k / d_k = ucol2[k] / N^2,   rows: B_k / d_k = urow2d[k] / (N^2 d_k).
template <int KIND, int N>
__device__ __forceinline__ float basis_factor(int k, int basis) {
  const TransformInfo<N>& I = info<KIND, N>();
  constexpr float inv_n2 = 1.0f / static_cast<float>(N * N);
  return basis == ADCT_BASIS_COLS
             ? static_cast<float>(I.ucol2[k]) * inv_n2
             : static_cast<float>(I.urow2d[k]) / static_cast<float>(I.d[k]) * inv_n2;
}

// ------------------------------------------------------------------ moments
struct MomParams {
  const void* src;
  Geom g;
  unsigned long long* mom;   // [batch][moment_words(N)]
  int wpi;                   // workgroups per image
};

// Every |b| of 8-bit input is at most 128 l1max^2; when that is below 2^15
// the square fits a 24-bit multiply and has no high half.
template <int KIND, int N, int DT>
constexpr bool small_squares() {
  constexpr TransformInfo<N> I = make_info<KIND, N>();
  return DT == DT_U8 && 128 * I.l1max * I.l1max < 32768;
}

template <int KIND, int N, int DT>
__global__ __launch_bounds__(kBlock) void moments_kernel(MomParams p) {
  static_assert(N >= 16, "8 x 8 tiles: moments8_kernel");
  using C = Cfg<N>;
  constexpr int NN = N * N;
  constexpr int PPT = NN >= kBlock ? NN / kBlock : 1;      // positions per thread
  constexpr int KSTEP = NN >= kBlock ? 1 : kBlock / NN;    // tiles between a thread's tiles
  constexpr bool SMALL = small_squares<KIND, N, DT>();
  constexpr int RED = KSTEP > 1 ? 6 * kBlock : 0;          // int words of the N = 8 reduction
  __shared__ __align__(16) int S[C::WORDS > RED ? C::WORDS : RED];
  __shared__ long long red_a[kBlock / 64][2];

  const int img = blockIdx.y;
  const int t = threadIdx.x;
  const int a_idx = t / C::TPW, k = t % C::TPW;
  const int groups_x = (p.g.tiles_x + C::TPW - 1) / C::TPW;
  const int64_t groups = static_cast<int64_t>(groups_x) * p.g.tiles_y;
  const int p0 = NN >= kBlock ? t : t % NN;
  const int k0 = NN >= kBlock ? 0 : t / NN;

  long long s1[PPT];
  unsigned long long s2lo[PPT], s2hi[PPT];
#pragma unroll
  for (int q = 0; q < PPT; ++q) {
    s1[q] = 0;
    s2lo[q] = 0;
    s2hi[q] = 0;
  }
  long long a1 = 0;
  unsigned long long a2 = 0;
  long long tiles = 0;

  // U tile groups per step, q0 + u wpi (u < U): their rows are all loaded
  // before the first is transformed, so a workgroup keeps U row loads in
  // flight (the walk covers the image's groups b, b + wpi, ... exactly once)
  constexpr int U = N == 16 ? 2 : 1;
  for (int64_t q0 = blockIdx.x; q0 < groups; q0 += static_cast<int64_t>(U) * p.wpi) {
    RowWords<N, DT> xs[U];
    int nacts[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t q = q0 + static_cast<int64_t>(u) * p.wpi;
      nacts[u] = 0;
      int64_t pix = 0;
      if (q < groups) {
        const int ty = static_cast<int>(q / groups_x);
        const int tx0 = static_cast<int>(q - static_cast<int64_t>(ty) * groups_x) * C::TPW;
        nacts[u] = min(C::TPW, p.g.tiles_x - tx0);
        pix = static_cast<int64_t>(img) * p.g.image_stride +
              static_cast<int64_t>(ty) * N * p.g.pitch + static_cast<int64_t>(tx0 + k) * N;
      }
      load_row<N, DT>(p.src, pix + static_cast<int64_t>(a_idx) * p.g.pitch, k < nacts[u], xs[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int nact = nacts[u];
      if (nact == 0) break;   // uniform: the walk's last groups
      const RowWords<N, DT>& x = xs[u];
      {   // row transform into the column-major exchange area
        int a[N];
        unpack_row<N, DT>(x, a);
        fwdN<KIND, N>(a);
#pragma unroll
        for (int j = 0; j < N; ++j) S[k * C::TS + j * C::CS + a_idx] = a[j];
      }
      if (k < nact) {   // pixel sums of this row, level-shifted for 8-bit input
        if constexpr (DT == DT_U8) {
          uint32_t sx = 0, sxx = 0;
#pragma unroll
          for (int d = 0; d < RowWords<N, DT>::W; ++d) {
            sx = __builtin_amdgcn_udot4(x.w[d], 0x01010101u, sx, false);
            sxx = __builtin_amdgcn_udot4(x.w[d], x.w[d], sxx, false);
          }
          // a = x - 128: sum a = sum x - 128 N, sum a^2 = sum x^2 - 256 sum x + 128^2 N
          a1 += static_cast<long long>(sx) - 128 * N;
          a2 += static_cast<unsigned long long>(sxx) + 16384ull * N - 256ull * sx;
        } else {
          int xv[N];
          unpack_row<N, DT>(x, xv);
#pragma unroll
          for (int i = 0; i < N; ++i) {
            a1 += xv[i];
            a2 += static_cast<unsigned long long>(static_cast<long long>(xv[i]) * xv[i]);
          }
        }
      }
      __syncthreads();
      int c[N];
      read_column<N, kBlock>(S, a_idx, k, c);
      fwdN<KIND, N>(c);
      if constexpr (DT == DT_U8)
        if (a_idx == 0) c[0] -= 128 * N * N;   // level shift folded into the DC coefficient
      __syncthreads();
      write_column_rows<N, kBlock>(S, a_idx, k, c);   // [k][v][u], row stride ZS
      __syncthreads();
#pragma unroll
      for (int pq = 0; pq < PPT; ++pq) {
        const int pos = p0 + pq * kBlock;
        const int off = (pos / N) * C::ZS + pos % N;
        for (int kk = k0; kk < nact; kk += KSTEP) {
          const int b = S[kk * C::TS + off];
          s1[pq] += b;
          if constexpr (SMALL) {
            s2lo[pq] += static_cast<uint32_t>(__mul24(b, b));
          } else {
            const unsigned long long sq =
                static_cast<unsigned long long>(static_cast<long long>(b) * b);
            s2lo[pq] += static_cast<uint32_t>(sq);
            s2hi[pq] += sq >> 32;
          }
        }
      }
      tiles += nact;
      __syncthreads();   // S is rewritten by the next group
    }
  }

  unsigned long long* rec = p.mom + static_cast<int64_t>(img) * (3 * NN + 4);
  if constexpr (KSTEP > 1) {
    // N = 8: threads t, t + 64, t + 128, t + 192 hold the same position
    unsigned long long* R = reinterpret_cast<unsigned long long*>(S);
    R[t] = static_cast<unsigned long long>(s1[0]);
    R[kBlock + t] = s2lo[0];
    R[2 * kBlock + t] = s2hi[0];
    __syncthreads();
    if (t < NN) {
      unsigned long long v1 = 0, vlo = 0, vhi = 0;
#pragma unroll
      for (int m = 0; m < KSTEP; ++m) {
        v1 += R[t + m * NN];
        vlo += R[kBlock + t + m * NN];
        vhi += R[2 * kBlock + t + m * NN];
      }
      if (v1 != 0) atomicAdd(rec + t, v1);
      if (vlo != 0) atomicAdd(rec + NN + t, vlo);
      if (vhi != 0) atomicAdd(rec + 2 * NN + t, vhi);
    }
  } else {
#pragma unroll
    for (int pq = 0; pq < PPT; ++pq) {
      const int pos = p0 + pq * kBlock;
      if (s1[pq] != 0) atomicAdd(rec + pos, static_cast<unsigned long long>(s1[pq]));
      if (s2lo[pq] != 0) atomicAdd(rec + NN + pos, s2lo[pq]);
      if (s2hi[pq] != 0) atomicAdd(rec + 2 * NN + pos, s2hi[pq]);
    }
  }
  // pixel sums: wave, then workgroup
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a1 += __shfl_xor(a1, off, 64);
    a2 += __shfl_xor(a2, off, 64);
  }
  if ((t & 63) == 0) {
    red_a[t >> 6][0] = a1;
    red_a[t >> 6][1] = static_cast<long long>(a2);
  }
  __syncthreads();
  if (t == 0 && tiles > 0) {
    long long b1 = 0;
    unsigned long long b2 = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      b1 += red_a[w][0];
      b2 += static_cast<unsigned long long>(red_a[w][1]);
    }
    atomicAdd(rec + 3 * NN, static_cast<unsigned long long>(tiles));
    atomicAdd(rec + 3 * NN + 1, static_cast<unsigned long long>(tiles) * NN);
    if (b1 != 0) atomicAdd(rec + 3 * NN + 2, static_cast<unsigned long long>(b1));
    if (b2 != 0) atomicAdd(rec + 3 * NN + 3, b2);
  }
}

// 8 x 8 tiles of int16 images (8-bit input takes moments8_mfma): one thread
// per tile, one wave per workgroup (as the fused 8-point kernels).  A wave
// walks the 64-tile groups q = b, b + wpi, ... of its image; for each it
// transforms its tiles in registers, writes the 64 coefficients of each tile
// to LDS, and lane p then adds position p of all the group's tiles to its
// running sums, squares split into 32-bit halves summed in 64 bits.  One set
// of atomics per wave at the end.
template <int KIND>
__global__ __launch_bounds__(t8::kWave) void moments8_kernel(MomParams p) {
  using namespace t8;
  constexpr int DT = DT_I16;
  constexpr int NN = kN * kN;
  constexpr int RS = NN + 1;
  __shared__ int lds[kWave * RS];
  const int img = blockIdx.y;
  const int lane = threadIdx.x;
  const int groups_x = (p.g.tiles_x + kWave - 1) / kWave;
  const int64_t groups = static_cast<int64_t>(groups_x) * p.g.tiles_y;
  long long s1 = 0, a1 = 0;
  unsigned long long s2lo = 0, s2hi = 0, a2 = 0;
  long long tiles = 0;
  for (int64_t q = blockIdx.x; q < groups; q += p.wpi) {
    const int ty = static_cast<int>(q / groups_x);
    const int gx = static_cast<int>(q - static_cast<int64_t>(ty) * groups_x);
    const WaveTiles w = wave_tiles_at(p.g, gx, ty, img);
    Raw<DT> raw;
    load_raw<DT>(p.src, w.pix, p.g.pitch, w.active, raw);
    int a[kN][kN];
    unpack<DT>(raw, a);
    if (w.active) {   // pixel sums of the tile
#pragma unroll
      for (int i = 0; i < kN; ++i)
#pragma unroll
        for (int j = 0; j < kN; ++j) {
          a1 += a[i][j];
          a2 += static_cast<unsigned long long>(static_cast<long long>(a[i][j]) * a[i][j]);
        }
    }
    forward2d<KIND>(a);
#pragma unroll
    for (int v = 0; v < kN; ++v)
#pragma unroll
      for (int u = 0; u < kN; ++u) lds[lane * RS + v * kN + u] = a[v][u];
    __syncthreads();
    // lane = coefficient position; tiles of the group one after the other
    for (int t = 0; t < w.nact; ++t) {
      const int b = lds[t * RS + lane];
      s1 += b;
      const unsigned long long sq = static_cast<unsigned long long>(static_cast<long long>(b) * b);
      s2lo += static_cast<uint32_t>(sq);
      s2hi += sq >> 32;
    }
    tiles += w.nact;
    __syncthreads();   // the next group rewrites the LDS area
  }
  unsigned long long* rec = p.mom + static_cast<int64_t>(img) * (3 * NN + 4);
  if (s1 != 0) atomicAdd(rec + lane, static_cast<unsigned long long>(s1));
  if (s2lo != 0) atomicAdd(rec + NN + lane, s2lo);
  if (s2hi != 0) atomicAdd(rec + 2 * NN + lane, s2hi);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a1 += __shfl_xor(a1, off, 64);
    a2 += __shfl_xor(a2, off, 64);
  }
  if (lane == 0 && tiles > 0) {
    atomicAdd(rec + 3 * NN, static_cast<unsigned long long>(tiles));
    atomicAdd(rec + 3 * NN + 1, static_cast<unsigned long long>(tiles) * NN);
    if (a1 != 0) atomicAdd(rec + 3 * NN + 2, static_cast<unsigned long long>(a1));
    if (a2 != 0) atomicAdd(rec + 3 * NN + 3, a2);
  }
}

// 8 x 8 tiles of 8-bit images on the int8 matrix cores.  With vec(A) the 64
// pixels of a tile in row-major order, vec(B) = (T (x) T) vec(A - 128); the
// entries of T lie in {0, +-1, +-2}, so T (x) T and A - 128 (a byte XOR with
// 0x80) are int8 operands and the int32 products are exact.  One
// v_mfma_i32_16x16x64_i8 multiplies 16 rows of T (x) T (lane l: row l % 16,
// pixels 16 (l / 16) .. + 15) by the pixels of 16 tiles (lane l: rows
// 2 (l / 16), 2 (l / 16) + 1 of tile l % 16), and lane l receives coefficient
// 16 blk + 4 (l / 16) + t of tile l % 16 in accumulator t of block blk.
// A wave walks the 64-tile groups q = b, b + wpi, ... of its image (four
// 16-tile steps, 512 B per pixel row, as the butterfly kernel).  Each lane
// adds its 16 coefficients and their squares to 32-bit run sums; every RUN
// groups the wave folds the run sums through LDS into 64-bit totals, lane p
// owning coefficient position p.  The transform costs the vector units
// nothing, which leaves about 3 VALU instructions per pixel (run sums,
// pixel sums, operand bytes) against about 11 in moments8_kernel.
typedef int v4i_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint32_t pack_i8x4(int a, int b, int c, int d) {
  return (static_cast<uint32_t>(a) & 0xffu) | ((static_cast<uint32_t>(b) & 0xffu) << 8) |
         ((static_cast<uint32_t>(c) & 0xffu) << 16) | (static_cast<uint32_t>(d) << 24);
}

// Five waves per SIMD: the compiler then keeps the accumulators in 90
// VGPRs (no AGPRs, no spills) instead of 84 + 20, and the extra resident
// waves keep more pixel rows in flight (0.975 -> 0.83 ms per 4 GiB pass).
// One 4.3 KB fold buffer (sums, then squares) lets LDS hold 36 one-wave
// workgroups per compute unit, so the registers set the limit (20).
template <int KIND>
__global__ __launch_bounds__(t8::kWave) __attribute__((amdgpu_waves_per_eu(5)))
void moments8_mfma(MomParams p) {
  using namespace t8;
  constexpr int NN = kN * kN;
  constexpr TransformInfo<8> kInf = make_info<KIND, 8>();
  constexpr unsigned long long kBmax = 128ull * kInf.l1max * kInf.l1max;   // largest |b|
  static_assert(kBmax < (1u << 15), "squares of 24-bit products");
  // groups per run: a lane adds 4 squares per group, and a run's sum of
  // squares must stay below 2^32
  constexpr int RUN = 4ull * 8 * kBmax * kBmax < (1ull << 32)   ? 8
                      : 4ull * 4 * kBmax * kBmax < (1ull << 32) ? 4
                      : 4ull * 2 * kBmax * kBmax < (1ull << 32) ? 2 : 1;
  constexpr int FS = 17;   // LDS stride of a lane's 16 run sums
  __shared__ int fold[kWave * FS];   // the sums, then the squares
  const TransformInfo<8>& I = info<KIND, 8>();
  const int lane = threadIdx.x;
  const int q = lane >> 4, col = lane & 15;

  // rows 16 blk .. 16 blk + 15 of T (x) T as the A operand of block blk
  v4i_t fa[4];
#pragma unroll
  for (int blk = 0; blk < 4; ++blk) {
    const int v = 2 * blk + (col >> 3), u = col & 7;
    uint32_t w4[4];
#pragma unroll
    for (int w = 0; w < 4; ++w) {
      int f[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int b = 4 * w + e;
        f[e] = I.t[v][2 * q + (b >> 3)] * I.t[u][b & 7];
      }
      w4[w] = pack_i8x4(f[0], f[1], f[2], f[3]);
    }
    fa[blk] = v4i_t{static_cast<int>(w4[0]), static_cast<int>(w4[1]), static_cast<int>(w4[2]),
                    static_cast<int>(w4[3])};
  }

  const int img = blockIdx.y;
  const int groups_x = (p.g.tiles_x + 63) / 64;
  const int64_t groups = static_cast<int64_t>(groups_x) * p.g.tiles_y;
  const uint8_t* src = static_cast<const uint8_t*>(p.src) + static_cast<int64_t>(img) * p.g.image_stride;
  const v4i_t zero = {0, 0, 0, 0};
  // run sums: coefficients accumulated by the matrix cores themselves (the
  // accumulator operand), squares by the vector units
  v4i_t s1r[4] = {zero, zero, zero, zero};
  uint32_t s2r[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) s2r[k] = 0;
  long long t1 = 0, a1 = 0;             // t1, t2: totals of coefficient position `lane`
  unsigned long long t2 = 0, a2 = 0;
  long long tiles = 0;

  // the lanes holding position `lane`: 16 (lane >> 2 & 3) + c, sum slot k
  const int pk = 4 * (lane >> 4) + (lane & 3);
  const int ph = 16 * ((lane >> 2) & 3);
  auto fold_run = [&]() {
#pragma unroll
    for (int k = 0; k < 16; ++k) fold[lane * FS + k] = s1r[k >> 2][k & 3];
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) s1r[blk] = zero;
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) t1 += fold[(ph + c) * FS + pk];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      fold[lane * FS + k] = static_cast<int>(s2r[k]);
      s2r[k] = 0;
    }
    __syncthreads();
#pragma unroll
    for (int c = 0; c < 16; ++c) t2 += static_cast<uint32_t>(fold[(ph + c) * FS + pk]);
    __syncthreads();
  };

  // the wave's 16-tile steps, four per group, with the rows of the next two
  // steps in flight while a step is computed.  A cursor (tile row, group
  // column, step) walks the groups blockIdx.x, + wpi, ... without divisions.
  const int64_t my_groups = blockIdx.x < groups ? (groups - 1 - blockIdx.x) / p.wpi + 1 : 0;
  const int64_t nsteps = 4 * my_groups;
  const int dty = p.wpi / groups_x, dgx = p.wpi - dty * groups_x;
  int cy = static_cast<int>(blockIdx.x) / groups_x;
  int cx = static_cast<int>(blockIdx.x) - cy * groups_x;
  int cj = 0;
  auto load_step = [&](uint2& a, uint2& b) {   // rows 2q, 2q + 1 of the cursor's tile
    const int tile = 64 * cx + 16 * cj + col;
    a = make_uint2(0x80808080u, 0x80808080u);
    b = a;
    if (tile < p.g.tiles_x) {
      const uint8_t* x = src + static_cast<int64_t>(8 * cy + 2 * q) * p.g.pitch +
                         static_cast<int64_t>(tile) * 8;
      a = ld_global(reinterpret_cast<const uint2*>(x));
      b = ld_global(reinterpret_cast<const uint2*>(x + p.g.pitch));
    }
  };
  // two steps in flight: (n0, n1) holds step i + 1 and (m0, m1) step i + 2
  // when step i is computed; the cursor stands at the step to load next, and
  // (ux, uj) at the step computed
  int ux = cx, uj = 0;
  auto advance = [&]() {
    if (++cj == 4) {
      cj = 0;
      cx += dgx;
      cy += dty;
      if (cx >= groups_x) {
        cx -= groups_x;
        ++cy;
      }
    }
  };
  uint2 n0 = make_uint2(0x80808080u, 0x80808080u), n1 = n0, m0 = n0, m1 = n0;
  if (nsteps > 0) load_step(n0, n1);
  advance();
  if (nsteps > 1) load_step(m0, m1);
  advance();
  int run = 0;
  for (int64_t i = 0; i < nsteps; ++i) {
    const uint2 r0 = n0, r1 = n1;
    n0 = m0;
    n1 = m1;
    const int tx0 = 64 * ux;
    const bool active = tx0 + 16 * uj + col < p.g.tiles_x;
    const bool last = uj == 3;
    if (++uj == 4) {
      uj = 0;
      ux += dgx;
      if (ux >= groups_x) ux -= groups_x;
    }
    if (i + 2 < nsteps) load_step(m0, m1);
    advance();
    if (active) {   // pixel sums of the two rows, level-shifted
      uint32_t sx = 0, sxx = 0;
      const uint32_t ws[4] = {r0.x, r0.y, r1.x, r1.y};
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        sx = __builtin_amdgcn_udot4(ws[k], 0x01010101u, sx, false);
        sxx = __builtin_amdgcn_udot4(ws[k], ws[k], sxx, false);
      }
      a1 += static_cast<long long>(sx) - 128 * 16;
      a2 += static_cast<unsigned long long>(sxx) + 16384ull * 16 - 256ull * sx;
    }
    const v4i_t px = {static_cast<int>(r0.x ^ 0x80808080u), static_cast<int>(r0.y ^ 0x80808080u),
                      static_cast<int>(r1.x ^ 0x80808080u), static_cast<int>(r1.y ^ 0x80808080u)};
#pragma unroll
    for (int blk = 0; blk < 4; ++blk) {
      const v4i_t d = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[blk], px, zero, 0, 0, 0);
      s1r[blk] = __builtin_amdgcn_mfma_i32_16x16x64_i8(fa[blk], px, s1r[blk], 0, 0, 0);
#pragma unroll
      for (int t = 0; t < 4; ++t) s2r[4 * blk + t] += static_cast<uint32_t>(__mul24(d[t], d[t]));
    }
    if (last) {   // end of a group (uniform: every lane walks the same steps)
      tiles += min(64, p.g.tiles_x - tx0);
      if (++run == RUN) {
        fold_run();
        run = 0;
      }
    }
  }
  if (run > 0) fold_run();
  unsigned long long* rec = p.mom + static_cast<int64_t>(img) * (3 * NN + 4);
  if (t1 != 0) atomicAdd(rec + lane, static_cast<unsigned long long>(t1));
  if (t2 != 0) atomicAdd(rec + NN + lane, t2);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a1 += __shfl_xor(a1, off, 64);
    a2 += __shfl_xor(a2, off, 64);
  }
  if (lane == 0 && tiles > 0) {
    atomicAdd(rec + 3 * NN, static_cast<unsigned long long>(tiles));
    atomicAdd(rec + 3 * NN + 1, static_cast<unsigned long long>(tiles) * NN);
    if (a1 != 0) atomicAdd(rec + 3 * NN + 2, static_cast<unsigned long long>(a1));
    if (a2 != 0) atomicAdd(rec + 3 * NN + 3, a2);
  }
}

// ----------------------------------------------------- measured coding gain
// count * s2 - s1^2 = count^2 times the population variance, exactly (128-bit)
__device__ __forceinline__ float scaled_variance(unsigned long long count, unsigned long long s2lo,
                                                 unsigned long long s2hi, long long s1) {
  const unsigned __int128 s2 = (static_cast<unsigned __int128>(s2hi) << 32) + s2lo;
  const unsigned long long m = static_cast<unsigned long long>(s1 < 0 ? -s1 : s1);
  const unsigned __int128 v = static_cast<unsigned __int128>(count) * s2 -
                              static_cast<unsigned __int128>(m) * m;
  const float hi = static_cast<float>(static_cast<unsigned long long>(v >> 64));
  const float lo = static_cast<float>(static_cast<unsigned long long>(v));
  return fmaf(hi, 18446744073709551616.0f, lo);
}

// One workgroup per record.  A_vu B_v B_u = (var_b / var_x) f_v f_u with
// f the basis factors above; the gain is -10/N^2 sum log10 of that.
template <int KIND, int N>
__global__ __launch_bounds__(kBlock) void coding_gain_kernel(const unsigned long long* mom,
                                                             int basis, float* cg) {
  constexpr int NN = N * N;
  __shared__ float red[kBlock / 64];
  __shared__ int zero_var[kBlock / 64];
  const unsigned long long* rec = mom + static_cast<int64_t>(blockIdx.x) * (3 * NN + 4);
  const unsigned long long tiles = rec[3 * NN], pixels = rec[3 * NN + 1];
  const float vx = scaled_variance(pixels, rec[3 * NN + 3], 0ull, static_cast<long long>(rec[3 * NN + 2]));
  const float fp = static_cast<float>(pixels), ft = static_cast<float>(tiles);
  // var_b / var_x = (Vb / tiles^2) / (Vx / pixels^2)
  const float ratio = (fp / ft) * (fp / ft) / vx;
  float sum = 0.0f;
  int zeros = 0;
  for (int pos = threadIdx.x; pos < NN; pos += kBlock) {
    const float vb = scaled_variance(tiles, rec[NN + pos], rec[2 * NN + pos],
                                     static_cast<long long>(rec[pos]));
    if (vb == 0.0f) ++zeros;
    else sum += log10f(vb * ratio * (basis_factor<KIND, N>(pos / N, basis) *
                                     basis_factor<KIND, N>(pos % N, basis)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    sum += __shfl_xor(sum, off, 64);
    zeros += __shfl_xor(zeros, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    red[threadIdx.x >> 6] = sum;
    zero_var[threadIdx.x >> 6] = zeros;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    float s = 0.0f;
    int z = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
      s += red[w];
      z += zero_var[w];
    }
    float g;
    if (tiles == 0 || vx == 0.0f) g = __builtin_nanf("");
    else if (z > 0) g = INFINITY;
    else g = -10.0f / static_cast<float>(NN) * s;
    cg[blockIdx.x] = g;
  }
}

// ------------------------------------------------- AR(1) model coding gain
// One wave per correlation value rho; lane k < N evaluates A_k B_k.  With
// h row k of T, h R h^T for R[m][n] = rho^|m-n| is evaluated in the
// innovations form of the first-order Markov process (x_0 = w_0,
// x_n = rho x_(n-1) + sqrt(1 - rho^2) w_n): with z_j = sum_(n>=j) rho^(n-j) h_n,
//   h R h^T = z_0^2 + (1 - rho^2) sum_(j>=1) z_j^2,
// a sum of non-negative terms, which stays accurate as rho -> 1 where the
// entries of R nearly cancel against the zero-sum AC rows.  The KLT's gain
// is -10/N log10 det R with det R = (1 - rho^2)^(N-1).
template <int KIND, int N>
__global__ __launch_bounds__(64) void coding_gain_ar1_kernel(const float* rho, int count,
                                                             int basis, float* cg, float* cg_klt) {
  const int i = blockIdx.x;
  const int k = threadIdx.x;
  const float r = rho[i];
  float term = 0.0f;
  if (k < N) {
    const TransformInfo<N>& I = info<KIND, N>();
    float z = 0.0f, acc = 0.0f;
    for (int n = N - 1; n >= 1; --n) {
      z = fmaf(r, z, static_cast<float>(I.t[k][n]));
      acc = fmaf(z, z, acc);
    }
    z = fmaf(r, z, static_cast<float>(I.t[k][0]));
    const float one_minus_r2 = (1.0f - r) * (1.0f + r);
    const float hrh = fmaf(one_minus_r2, acc, z * z);
    term = log10f(hrh * basis_factor<KIND, N>(k, basis));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) term += __shfl_xor(term, off, 64);
  if (k == 0) {
    if (cg != nullptr) cg[i] = -10.0f / static_cast<float>(N) * term;
    if (cg_klt != nullptr)
      cg_klt[i] = -10.0f * static_cast<float>(N - 1) / static_cast<float>(N) *
                  (log1pf(-r * r) * 0.43429448190325182f);
  }
}

// -------------------------------------------------------------- workspace
__global__ void fill_zero_u64(unsigned long long* p, int64_t n) {
  for (int64_t i = blockIdx.x * static_cast<int64_t>(blockDim.x) + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    p[i] = 0ull;
}

// -------------------------------------------------------------------- PSNR
__global__ void psnr_plain_kernel(const unsigned long long* sse, int count, float npix, float* psnr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const unsigned long long e = sse[i];
  psnr[i] = e == 0ull ? INFINITY : 10.0f * log10f(65025.0f * npix / static_cast<float>(e));
}

template <int KIND, int N>
hipError_t launch_moments_typed(int dtype, const MomParams& p, hipStream_t s) {
  const dim3 grid(p.wpi, p.g.batch);
  if (dtype == DT_U8) moments_kernel<KIND, N, DT_U8><<<grid, kBlock, 0, s>>>(p);
  else moments_kernel<KIND, N, DT_I16><<<grid, kBlock, 0, s>>>(p);
  return hipGetLastError();
}

template <int KIND>
hipError_t launch_cg_typed(int n, const unsigned long long* mom, int count, int basis, float* cg,
                           hipStream_t s) {
  if (n == 8) coding_gain_kernel<KIND, 8><<<count, kBlock, 0, s>>>(mom, basis, cg);
  else if (n == 16) coding_gain_kernel<KIND, 16><<<count, kBlock, 0, s>>>(mom, basis, cg);
  else if (n == 32) coding_gain_kernel<KIND, 32><<<count, kBlock, 0, s>>>(mom, basis, cg);
  else coding_gain_kernel<KIND, 64><<<count, kBlock, 0, s>>>(mom, basis, cg);
  return hipGetLastError();
}

template <int KIND>
hipError_t launch_ar1_typed(int n, const float* rho, int count, int basis, float* cg,
                            float* cg_klt, hipStream_t s) {
  if (n == 8) coding_gain_ar1_kernel<KIND, 8><<<count, 64, 0, s>>>(rho, count, basis, cg, cg_klt);
  else if (n == 16) coding_gain_ar1_kernel<KIND, 16><<<count, 64, 0, s>>>(rho, count, basis, cg, cg_klt);
  else if (n == 32) coding_gain_ar1_kernel<KIND, 32><<<count, 64, 0, s>>>(rho, count, basis, cg, cg_klt);
  else coding_gain_ar1_kernel<KIND, 64><<<count, 64, 0, s>>>(rho, count, basis, cg, cg_klt);
  return hipGetLastError();
}

}  // namespace

int launch_moments(int kind, int n, int dtype, const void* src, const Geom& g,
                   unsigned long long* mom, hipStream_t s) {
  MomParams p;
  p.src = src;
  p.g = g;
  p.mom = mom;
  if (n == 8) {
    // one-wave workgroups, about 32768 in all (several times what the chip
    // holds at once, so the last ones to start leave little tail), each
    // walking 64-tile groups of its image: 8-bit input on the matrix cores,
    // int16 on the butterflies
    const int64_t groups8 = static_cast<int64_t>((g.tiles_x + 63) / 64) * g.tiles_y;
    int64_t wpi8 = (32768 + g.batch - 1) / g.batch;
    wpi8 = std::max<int64_t>(1, std::min<int64_t>(wpi8, groups8));
    p.wpi = static_cast<int>(wpi8);
    const dim3 grid8(p.wpi, g.batch);
    auto go = [&](auto kind_tag) {
      constexpr int K = decltype(kind_tag)::value;
      if (dtype == DT_U8) moments8_mfma<K><<<grid8, t8::kWave, 0, s>>>(p);
      else moments8_kernel<K><<<grid8, t8::kWave, 0, s>>>(p);
    };
    switch (kind) {
      case KIND_SIGN: go(std::integral_constant<int, KIND_SIGN>{}); break;
      case KIND_ROUND: go(std::integral_constant<int, KIND_ROUND>{}); break;
      case KIND_WHT: go(std::integral_constant<int, KIND_WHT>{}); break;
      case KIND_SDCT: go(std::integral_constant<int, KIND_SDCT>{}); break;
      default: go(std::integral_constant<int, KIND_HT>{}); break;
    }
    return hipGetLastError();
  }
  const int tpw = kBlock / n;
  const int64_t groups = static_cast<int64_t>((g.tiles_x + tpw - 1) / tpw) * g.tiles_y;
  // about 2048 workgroups in all (8 per CU), each walking its image's groups
  // with stride wpi; at least one group each
  int64_t wpi = (2048 + g.batch - 1) / g.batch;
  if (wpi > groups) wpi = groups;
  if (wpi < 1) wpi = 1;
  p.wpi = static_cast<int>(wpi);
  if (n == 64) {   // 8-bit input only (the host refuses the rest)
    const dim3 grid(p.wpi, p.g.batch);
    if (kind == KIND_SIGN) moments_kernel<KIND_SIGN, 64, DT_U8><<<grid, kBlock, 0, s>>>(p);
    else moments_kernel<KIND_ROUND, 64, DT_U8><<<grid, kBlock, 0, s>>>(p);
    return hipGetLastError();
  }
  if (kind == KIND_SIGN) {
    if (n == 16) return launch_moments_typed<KIND_SIGN, 16>(dtype, p, s);
    return launch_moments_typed<KIND_SIGN, 32>(dtype, p, s);
  }
  if (n == 16) return launch_moments_typed<KIND_ROUND, 16>(dtype, p, s);
  return launch_moments_typed<KIND_ROUND, 32>(dtype, p, s);
}

int launch_coding_gain(int kind, int n, int basis, const unsigned long long* mom, int count,
                       float* cg, hipStream_t s) {
  switch (kind) {
    case KIND_WHT: coding_gain_kernel<KIND_WHT, 8><<<count, kBlock, 0, s>>>(mom, basis, cg); break;
    case KIND_SDCT: coding_gain_kernel<KIND_SDCT, 8><<<count, kBlock, 0, s>>>(mom, basis, cg); break;
    case KIND_HT: coding_gain_kernel<KIND_HT, 8><<<count, kBlock, 0, s>>>(mom, basis, cg); break;
    case KIND_SIGN: return launch_cg_typed<KIND_SIGN>(n, mom, count, basis, cg, s);
    default: return launch_cg_typed<KIND_ROUND>(n, mom, count, basis, cg, s);
  }
  return hipGetLastError();
}

int launch_coding_gain_ar1(int kind, int n, int basis, const float* rho, int count, float* cg,
                           float* cg_klt, hipStream_t s) {
  switch (kind) {
    case KIND_WHT:
      coding_gain_ar1_kernel<KIND_WHT, 8><<<count, 64, 0, s>>>(rho, count, basis, cg, cg_klt);
      break;
    case KIND_SDCT:
      coding_gain_ar1_kernel<KIND_SDCT, 8><<<count, 64, 0, s>>>(rho, count, basis, cg, cg_klt);
      break;
    case KIND_HT:
      coding_gain_ar1_kernel<KIND_HT, 8><<<count, 64, 0, s>>>(rho, count, basis, cg, cg_klt);
      break;
    case KIND_SIGN: return launch_ar1_typed<KIND_SIGN>(n, rho, count, basis, cg, cg_klt, s);
    default: return launch_ar1_typed<KIND_ROUND>(n, rho, count, basis, cg, cg_klt, s);
  }
  return hipGetLastError();
}

int launch_fill_zero(unsigned long long* p, int64_t words, hipStream_t s) {
  if (words <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((words + 255) / 256, 4096);
  fill_zero_u64<<<static_cast<int>(blocks), 256, 0, s>>>(p, words);
  return hipGetLastError();
}

int launch_psnr(const unsigned long long* sse, int count, int64_t pixels, float* psnr,
                hipStream_t s) {
  psnr_plain_kernel<<<(count + 255) / 256, 256, 0, s>>>(sse, count, static_cast<float>(pixels), psnr);
  return hipGetLastError();
}

}  // namespace adct
