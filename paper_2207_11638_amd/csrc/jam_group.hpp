// Workgroup-level processing of 16 x 16 and 32 x 32 tiles (Chen-JAM
// transforms of section 6.1), shared by the plain kernels and the ragged
// batch kernel.
//
// A workgroup of 256 threads owns TPW = 256/N tiles k = 0..TPW-1, each at its
// own pixel offset.  Thread L plays two roles:
//   row role    (i = L / TPW, k = L % TPW): row i of tile k;
//   column role (j = L / TPW, k = L % TPW): column j of tile k.
// When the tiles are horizontally adjacent (plain kernels) the lanes of a
// wave cover whole tile rows, so every pixel load/store of a wave is a run of
// 256 B (uint8) or 512 B (int16) per image row.  Each 1D N-point butterfly
// runs on N values in one thread's registers; the row<->column exchange goes
// through LDS with a padded layout (column stride N+1, tile stride 2 or 4 mod
// 32 words) that keeps every LDS access of a half-wave on distinct banks.
#pragma once

#include "adct_internal.hpp"

namespace adct {
namespace jam {

// Smallest tile stride >= n * (n + 1) words that is congruent to `spread`
// modulo 32: the TPW tiles of a half-wave then start on banks `spread` apart.
constexpr int tile_stride(int n, int spread) {
  int ts = n * (n + 1);
  while (ts % 32 != spread) ++ts;
  return ts;
}

template <int N, int BS = 256>
struct Cfg {
  static constexpr int TPW = BS / N;                        // tiles per workgroup
  static constexpr int CS = N + 1;                          // LDS column stride (words)
  static constexpr int TS = tile_stride(N, 32 / TPW);       // LDS tile stride (words)
  static constexpr int WORDS = TPW * TS;
  static constexpr int LOG2N = N == 16 ? 4 : 5;
  static constexpr int SROUND = 2 + 2 * LOG2N;              // divide by 4 N^2
  static_assert(TPW >= 2 && TPW <= 32, "unsupported block size");
};

constexpr int kBlock = 256;
constexpr int kMaxWords = Cfg<32>::WORDS;

// Constant tables of one (transform, N, qstep), staged in LDS.
struct Shared {
  int32_t mq[16];
  int32_t dq[16];
  float s2[16];
  int32_t cls[32];
};

__device__ __forceinline__ void load_tables(Shared& sh, const Tables& t, int n) {
  const int i = threadIdx.x;
  if (i < 16) {
    sh.mq[i] = t.mq[i];
    sh.dq[i] = t.dq[i];
    sh.s2[i] = t.s2[i];
  }
  if (i < n) sh.cls[i] = t.cls[i];
}

// Where this thread's tile lives and where the group's outputs go.
struct GroupIO {
  const void* src;
  void* dst;                  // reconstruction base (nullable)
  int64_t pitch;              // pixels
  int64_t tile_pix;           // pixel offset of tile k (this thread's k)
  bool active;                // tile k exists
  int nact;                   // number of tiles (k < nact exist)
  int r;                      // retained coefficients per tile
  int32_t* kept;              // [nact][r] block of this group (nullable)
  float* scaled;              // [nact][r] block of this group (nullable)
  unsigned long long* sse;    // error-energy accumulator of the group's image (nullable)
};

// ------------------------------------------------------------- pixel rows
template <int N, int DT>
__device__ __forceinline__ void load_row(const void* src, int64_t off, bool active, int (&x)[N]) {
  if constexpr (DT == DT_U8) {
    constexpr int V = N / 16;  // uint4 per row
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint8_t*>(src) + off);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      uint4 w = make_uint4(0x80808080u, 0x80808080u, 0x80808080u, 0x80808080u);
      if (active) w = p[q];
      const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int d = 0; d < 4; ++d)
#pragma unroll
        for (int b = 0; b < 4; ++b) x[16 * q + 4 * d + b] = (ws[d] >> (8 * b)) & 0xff;
    }
  } else {
    constexpr int V = N / 8;
    const uint4* p = reinterpret_cast<const uint4*>(static_cast<const int16_t*>(src) + off);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      uint4 w = make_uint4(0u, 0u, 0u, 0u);
      if (active) w = p[q];
      const uint32_t ws[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
      for (int d = 0; d < 4; ++d) {
        x[8 * q + 2 * d] = static_cast<int>(ws[d] << 16) >> 16;
        x[8 * q + 2 * d + 1] = static_cast<int>(ws[d]) >> 16;
      }
    }
  }
}

// Round z / 2^S half away from zero, clip, store one row; return its squared
// error against the original row x (when x is given).
template <int N, int DT, int S>
__device__ __forceinline__ unsigned long long store_row(void* dst, int64_t off, bool active,
                                                        const int (&z)[N], const int* x) {
  int y[N];
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if constexpr (DT == DT_U8)
      y[j] = round_shift_u8<S>(z[j]);
    else
      y[j] = min(max(round_shift<S>(z[j]), -32768), 32767);
  }
  unsigned long long err = 0;
  if (x != nullptr) {
    if constexpr (DT == DT_U8) {
      uint32_t acc = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const int d = y[j] - x[j];
        acc += static_cast<uint32_t>(__mul24(d, d));
      }
      err = acc;
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const long long d = y[j] - x[j];
        err += static_cast<unsigned long long>(d * d);
      }
    }
  }
  if (dst != nullptr && active) {
    if constexpr (DT == DT_U8) {
      uint4* p = reinterpret_cast<uint4*>(static_cast<uint8_t*>(dst) + off);
#pragma unroll
      for (int q = 0; q < N / 16; ++q) {
        uint32_t ws[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const int* yy = y + 16 * q + 4 * d;
          ws[d] = yy[0] | (yy[1] << 8) | (yy[2] << 16) | (yy[3] << 24);
        }
        st_stream(p + q, make_uint4(ws[0], ws[1], ws[2], ws[3]));
      }
    } else {
      uint4* p = reinterpret_cast<uint4*>(static_cast<int16_t*>(dst) + off);
#pragma unroll
      for (int q = 0; q < N / 8; ++q) {
        uint32_t ws[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) {
          const int* yy = y + 8 * q + 2 * d;
          ws[d] = (yy[0] & 0xffff) | (static_cast<uint32_t>(yy[1]) << 16);
        }
        st_stream(p + q, make_uint4(ws[0], ws[1], ws[2], ws[3]));
      }
    }
  }
  return err;
}

__device__ __forceinline__ int quantise(int b, int32_t mq) {
  const uint32_t mag = static_cast<uint32_t>(b < 0 ? -b : b);
  const uint64_t prod = static_cast<uint64_t>(mag) * static_cast<uint32_t>(mq) + (1ull << 23);
  const int lev = static_cast<int>(prod >> 24);
  return b < 0 ? -lev : lev;
}

// Wave-wide sum, one atomic per wave.
__device__ __forceinline__ void add_sse(unsigned long long* sse, unsigned long long e) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if ((threadIdx.x & 63) == 0 && e != 0) atomicAdd(sse, e);
}

// Number of rows kept in column u by the zig-zag prefix r (a prefix of the
// column: rows 0 .. count-1).
template <int N>
__device__ __forceinline__ int kept_rows(int u, int r) {
  int c = 0;
#pragma unroll
  for (int v = 0; v < N; ++v) c += zz_pos(N, v, u) < r ? 1 : 0;
  return c;
}

template <int N, int BS>
__device__ __forceinline__ void read_column(const int* S, int j, int k, int (&c)[N]) {
  using C = Cfg<N, BS>;
#pragma unroll
  for (int v = 0; v < N; ++v) c[v] = S[k * C::TS + j * C::CS + v];
}

template <int N, int BS>
__device__ __forceinline__ void write_column_rows(int* S, int j, int k, const int (&c)[N]) {
  using C = Cfg<N, BS>;
#pragma unroll
  for (int v = 0; v < N; ++v) S[k * C::TS + v * C::CS + j] = c[v];
}

template <int N, int BS>
__device__ __forceinline__ void read_row(const int* S, int i, int k, int (&z)[N]) {
  using C = Cfg<N, BS>;
#pragma unroll
  for (int u = 0; u < N; ++u) z[u] = S[k * C::TS + i * C::CS + u];
}

// Copy ``count`` contiguous words from LDS to global memory (all threads).
template <int BS>
__device__ __forceinline__ void copy_out(uint32_t* dst, const int* src, int count) {
  for (int e = threadIdx.x; e < count; e += BS) st_stream(dst + e, static_cast<uint32_t>(src[e]));
}

// Row forward: load row i of tile k, transform it, store it transposed so that
// column j of tile k is contiguous: S[k][j][i].  Returns the raw row in x.
template <int KIND, int N, int DT, int BS>
__device__ __forceinline__ void row_forward(int* S, const GroupIO& io, int i, int k, int (&x)[N]) {
  using C = Cfg<N, BS>;
  load_row<N, DT>(io.src, io.tile_pix + static_cast<int64_t>(i) * io.pitch, io.active, x);
  int a[N];
#pragma unroll
  for (int j = 0; j < N; ++j) a[j] = x[j];
  fwdN<KIND, N>(a);
#pragma unroll
  for (int j = 0; j < N; ++j) S[k * C::TS + j * C::CS + i] = a[j];
}

// ------------------------------------------------------------ fused group
// Forward -> retain / quantise -> (outputs) -> inverse -> round -> store -> SSE
// for the TPW tiles of one workgroup.  Every thread of the workgroup calls it.
template <int KIND, int N, int DT, bool QUANT, int BS = kBlock>
__device__ __forceinline__ void compress_group(int* S, const Shared& sh, const GroupIO& io) {
  using C = Cfg<N, BS>;
  const int a_idx = threadIdx.x / C::TPW;
  const int k = threadIdx.x % C::TPW;
  const int r = io.r;

  // phase 1: rows
  int x[N];
  row_forward<KIND, N, DT, BS>(S, io, a_idx, k, x);
  __syncthreads();

  // phase 2: columns, forward
  const int j = a_idx;
  int c[N];
  read_column<N, BS>(S, j, k, c);
  fwdN<KIND, N>(c);
  if constexpr (DT == DT_U8)
    if (j == 0) c[0] -= 128 * N * N;   // level shift folded into the DC coefficient
  const int keep = kept_rows<N>(j, r);
  const int cls_u = sh.cls[j];
  __syncthreads();  // S is free again

  // zig-zag outputs staged per tile as [k][pos] in S
  if (io.scaled != nullptr) {
#pragma unroll
    for (int v = 0; v < N; ++v)
      if (v < keep) {
        const float s = sh.s2[sh.cls[v] * 4 + cls_u];
        S[k * r + zz_pos(N, v, j)] = __builtin_bit_cast(int, static_cast<float>(c[v]) * s);
      }
    __syncthreads();
    copy_out<BS>(reinterpret_cast<uint32_t*>(io.scaled), S, io.nact * r);
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < N; ++v) {
    int b = v < keep ? c[v] : 0;
    if constexpr (QUANT) b = quantise(b, sh.mq[sh.cls[v] * 4 + cls_u]);
    c[v] = b;
  }
  if (io.kept != nullptr) {
#pragma unroll
    for (int v = 0; v < N; ++v)
      if (v < keep) S[k * r + zz_pos(N, v, j)] = c[v];
    __syncthreads();
    copy_out<BS>(reinterpret_cast<uint32_t*>(io.kept), S, io.nact * r);
    __syncthreads();
  }
  if (io.dst == nullptr && io.sse == nullptr) return;

  // phase 2b: columns, inverse
  if constexpr (QUANT) {
#pragma unroll
    for (int v = 0; v < N; ++v) c[v] = __mul24(c[v], sh.dq[sh.cls[v] * 4 + cls_u]);
  }
  invN<KIND, N>(c);
  if constexpr (QUANT) {
    // K = 2U: halve exactly so the second pass stays within 32 bits
#pragma unroll
    for (int v = 0; v < N; ++v) c[v] >>= 1;
  }
  write_column_rows<N, BS>(S, j, k, c);
  __syncthreads();

  // phase 3: rows, inverse
  const int i = a_idx;
  int z[N];
  read_row<N, BS>(S, i, k, z);
  invN<KIND, N>(z);
  // zonal: Z = 4 X, y = round(Z / (4 N^2)); quantised: Z = 2 X~, y = round(X~ / (2 N^2))
  const unsigned long long e = store_row<N, DT, C::SROUND>(
      io.dst, io.tile_pix + static_cast<int64_t>(i) * io.pitch, io.active, z,
      io.sse != nullptr ? x : nullptr);
  if (io.sse != nullptr) add_sse(io.sse, io.active ? e : 0ull);
  __syncthreads();  // S may be reused by the caller
}

}  // namespace jam
}  // namespace adct
