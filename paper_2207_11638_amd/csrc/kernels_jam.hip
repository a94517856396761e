// 16 x 16 and 32 x 32 kernels (Chen-JAM transforms of section 6.1).
//
// A workgroup of 256 threads owns 256/N horizontally adjacent tiles of one
// tile row.  Thread L plays two roles:
//   row role    (i = L / TPW, k = L % TPW): row i of tile k;
//   column role (j = L / TPW, k = L % TPW): column j of tile k.
// With this numbering the lanes of a wave cover whole tile rows, so every
// pixel load/store of a wave is a run of 256 B (uint8) or 512 B (int16) per
// image row.  Each 1D N-point butterfly runs on N values held in one
// thread's registers; the row<->column exchange goes through LDS with a
// padded layout (column stride N+1, tile stride = 2 or 4 mod 32 words) that
// keeps every LDS access of a half-wave on distinct banks.
//
//   fused:   load rows -> row forward -> LDS -> column forward -> retain /
//            quantise (+ zig-zag outputs staged through LDS for coalesced
//            stores) -> column inverse -> LDS -> row inverse -> round ->
//            store rows (+ error energy)
#include "adct_internal.hpp"

namespace adct {
namespace {

constexpr int kBlock = 256;

template <int N>
struct Cfg {
  static constexpr int TPW = kBlock / N;                    // tiles per workgroup
  static constexpr int CS = N + 1;                          // LDS column stride (words)
  static constexpr int TS = N == 16 ? 290 : 1060;           // LDS tile stride (words)
  static constexpr int WORDS = TPW * TS;
  static constexpr int LOG2N = N == 16 ? 4 : 5;
  static constexpr int SROUND = 2 + 2 * LOG2N;              // divide by 4 N^2
  static_assert(TS >= N * CS, "tile stride too small");
  static_assert(TS % 32 == (N == 16 ? 2 : 4), "tile stride breaks the bank spread");
};

struct Shared {
  int32_t mq[16];
  int32_t dq[16];
  float s2[16];
  int32_t cls[32];
  int32_t ccount[32];  // kept rows per column under the zig-zag prefix r
};

template <int N>
struct Place {
  int lane_a;  // i (row role) or j (column role)
  int k;       // tile within the workgroup
  int tx;      // tile column in the image
  bool active;
};

template <int N>
__device__ __forceinline__ Place<N> place() {
  using C = Cfg<N>;
  Place<N> pl;
  pl.lane_a = threadIdx.x / C::TPW;
  pl.k = threadIdx.x % C::TPW;
  return pl;
}

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

__device__ __forceinline__ void add_sse(unsigned long long* sse, int img, unsigned long long e) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
  if ((threadIdx.x & 63) == 0 && e != 0) atomicAdd(sse + img, e);
}

__device__ __forceinline__ void load_shared_tables(Shared& sh, const PassParams& p, int n) {
  const int t = threadIdx.x;
  if (t < 16) {
    sh.mq[t] = p.t.mq[t];
    sh.dq[t] = p.t.dq[t];
    sh.s2[t] = p.t.s2[t];
  }
  if (t < n) sh.cls[t] = p.t.cls[t];
}

// Number of rows kept in column u by the zig-zag prefix r.
template <int N>
__device__ __forceinline__ int kept_rows(int u, int r) {
  int c = 0;
#pragma unroll
  for (int v = 0; v < N; ++v) c += zz_pos(N, v, u) < r ? 1 : 0;
  return c;
}

// Geometry of the workgroup: first tile column, tile row, image.
struct WgPos {
  int tx0, ty, img;
  int64_t tile0;   // global index of tile k = 0
  int64_t pix0;    // pixel offset of the top-left corner of tile k = 0
};

template <int N>
__device__ __forceinline__ WgPos wg_pos(const Geom& g) {
  WgPos w;
  w.tx0 = blockIdx.x * Cfg<N>::TPW;
  w.ty = blockIdx.y;
  w.img = blockIdx.z;
  w.tile0 = (static_cast<int64_t>(w.img) * g.tiles_y + w.ty) * g.tiles_x + w.tx0;
  w.pix0 = static_cast<int64_t>(w.img) * g.image_stride +
           static_cast<int64_t>(w.ty) * N * g.pitch + static_cast<int64_t>(w.tx0) * N;
  return w;
}

// --------------------------------------------------------------- phases
// Row forward: load row i of tile k, transform it, store it transposed so
// that column j of tile k is contiguous: S[k][j][i].
template <int KIND, int N, int DT>
__device__ __forceinline__ void row_forward(int* S, const PassParams& p, const WgPos& w,
                                            int i, int k, bool active, int (&x)[N]) {
  using C = Cfg<N>;
  load_row<N, DT>(p.src, w.pix0 + static_cast<int64_t>(i) * p.g.pitch + k * N, active, x);
  int a[N];
#pragma unroll
  for (int j = 0; j < N; ++j) a[j] = x[j];
  fwdN<KIND, N>(a);
#pragma unroll
  for (int j = 0; j < N; ++j) S[k * C::TS + j * C::CS + i] = a[j];
}

// Column role: read column j of tile k from S[k][j][*].
template <int N>
__device__ __forceinline__ void read_column(const int* S, int j, int k, int (&c)[N]) {
  using C = Cfg<N>;
#pragma unroll
  for (int v = 0; v < N; ++v) c[v] = S[k * C::TS + j * C::CS + v];
}

// Column role: write column j of tile k as S[k][v][j] so rows are contiguous.
template <int N>
__device__ __forceinline__ void write_column_rows(int* S, int j, int k, const int (&c)[N]) {
  using C = Cfg<N>;
#pragma unroll
  for (int v = 0; v < N; ++v) S[k * C::TS + v * C::CS + j] = c[v];
}

template <int N>
__device__ __forceinline__ void read_row(const int* S, int i, int k, int (&z)[N]) {
  using C = Cfg<N>;
#pragma unroll
  for (int u = 0; u < N; ++u) z[u] = S[k * C::TS + i * C::CS + u];
}

// Copy ``count`` contiguous words from LDS to global memory (all threads).
template <typename T>
__device__ __forceinline__ void copy_out(T* dst, const int* src, int count) {
  uint32_t* d = reinterpret_cast<uint32_t*>(dst);
  for (int e = threadIdx.x; e < count; e += kBlock) st_stream(d + e, static_cast<uint32_t>(src[e]));
}

// ------------------------------------------------------------------ kernels
template <int KIND, int N, int DT, bool QUANT>
__global__ __launch_bounds__(kBlock) void compress_jam(PassParams p) {
  using C = Cfg<N>;
  __shared__ int S[C::WORDS];
  __shared__ Shared sh;
  load_shared_tables(sh, p, N);
  const WgPos w = wg_pos<N>(p.g);
  const int a_idx = threadIdx.x / C::TPW;
  const int k = threadIdx.x % C::TPW;
  const bool active = w.tx0 + k < p.g.tiles_x;
  const int nact = min(C::TPW, p.g.tiles_x - w.tx0);
  const int r = p.r;

  // phase 1: rows
  int x[N];
  row_forward<KIND, N, DT>(S, p, w, a_idx, k, active, x);
  __syncthreads();

  // phase 2: columns, forward
  const int j = a_idx;
  int c[N];
  read_column<N>(S, j, k, c);
  fwdN<KIND, N>(c);
  if constexpr (DT == DT_U8)
    if (j == 0) c[0] -= 128 * N * N;
  const int keep = kept_rows<N>(j, r);
  const int cls_u = sh.cls[j];
  __syncthreads();  // S is free again

  // zig-zag outputs staged per tile as [k][pos] in S
  if (p.scaled != nullptr) {
#pragma unroll
    for (int v = 0; v < N; ++v)
      if (v < keep) {
        const float s = sh.s2[sh.cls[v] * 4 + cls_u];
        S[k * r + zz_pos(N, v, j)] = __builtin_bit_cast(int, static_cast<float>(c[v]) * s);
      }
    __syncthreads();
    copy_out<float>(p.scaled + w.tile0 * r, S, nact * r);
    __syncthreads();
  }
#pragma unroll
  for (int v = 0; v < N; ++v) {
    int b = v < keep ? c[v] : 0;
    if constexpr (QUANT) b = quantise(b, sh.mq[sh.cls[v] * 4 + cls_u]);
    c[v] = b;
  }
  if (p.cout != nullptr) {
#pragma unroll
    for (int v = 0; v < N; ++v)
      if (v < keep) S[k * r + zz_pos(N, v, j)] = c[v];
    __syncthreads();
    copy_out<int32_t>(p.cout + w.tile0 * r, S, nact * r);
    __syncthreads();
  }
  if (p.dst == nullptr && p.sse == nullptr) return;

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
  write_column_rows<N>(S, j, k, c);
  __syncthreads();

  // phase 3: rows, inverse
  const int i = a_idx;
  int z[N];
  read_row<N>(S, i, k, z);
  invN<KIND, N>(z);
  // zonal: Z = 4 X, y = round(Z / (4 N^2)); quantised: Z = 2 X~, y = round(X~ / (2 N^2))
  const unsigned long long e = store_row<N, DT, C::SROUND>(
      p.dst, w.pix0 + static_cast<int64_t>(i) * p.g.pitch + k * N, active, z,
      p.sse != nullptr ? x : nullptr);
  if (p.sse != nullptr) add_sse(p.sse, w.img, active ? e : 0ull);
}

template <int KIND, int N, int DT>
__global__ __launch_bounds__(kBlock) void forward_jam(PassParams p) {
  using C = Cfg<N>;
  __shared__ int S[C::WORDS];
  const WgPos w = wg_pos<N>(p.g);
  const int a_idx = threadIdx.x / C::TPW;
  const int k = threadIdx.x % C::TPW;
  const bool active = w.tx0 + k < p.g.tiles_x;
  const int nact = min(C::TPW, p.g.tiles_x - w.tx0);
  int x[N];
  row_forward<KIND, N, DT>(S, p, w, a_idx, k, active, x);
  __syncthreads();
  const int j = a_idx;
  int c[N];
  read_column<N>(S, j, k, c);
  fwdN<KIND, N>(c);
  if constexpr (DT == DT_U8)
    if (j == 0) c[0] -= 128 * N * N;
  __syncthreads();
  // natural order within a tile, tiles contiguous: dense staging [k][v][u]
#pragma unroll
  for (int v = 0; v < N; ++v) S[k * N * N + v * N + j] = c[v];
  __syncthreads();
  copy_out<int32_t>(p.cout + w.tile0 * N * N, S, nact * N * N);
}

// Inverse from natural-order coefficients (DECOMP = false) or from the
// zig-zag-ordered retained coefficients of adct_compress (DECOMP = true).
template <int KIND, int N, int DT, bool QUANT, bool DECOMP>
__global__ __launch_bounds__(kBlock) void inverse_jam(PassParams p) {
  using C = Cfg<N>;
  __shared__ int S[C::WORDS];
  __shared__ Shared sh;
  load_shared_tables(sh, p, N);
  const WgPos w = wg_pos<N>(p.g);
  const int a_idx = threadIdx.x / C::TPW;
  const int k = threadIdx.x % C::TPW;
  const bool active = w.tx0 + k < p.g.tiles_x;
  const int nact = min(C::TPW, p.g.tiles_x - w.tx0);
  const int r = p.r;
  const int per_tile = DECOMP ? r : N * N;
  // stage this workgroup's coefficients, contiguous in global memory
  const int32_t* src = p.cin + w.tile0 * per_tile;
  for (int e = threadIdx.x; e < nact * per_tile; e += kBlock) S[e] = src[e];
  __syncthreads();
  const int j = a_idx;
  const int keep = kept_rows<N>(j, r);
  const int cls_u = sh.cls[j];
  int c[N];
#pragma unroll
  for (int v = 0; v < N; ++v) {
    int b = 0;
    if (v < keep && active)
      b = DECOMP ? S[k * r + zz_pos(N, v, j)] : S[k * N * N + v * N + j];
    if constexpr (QUANT) b = __mul24(b, sh.dq[sh.cls[v] * 4 + cls_u]);
    c[v] = b;
  }
  __syncthreads();
  invN<KIND, N>(c);
  if constexpr (QUANT) {
#pragma unroll
    for (int v = 0; v < N; ++v) c[v] >>= 1;
  }
  write_column_rows<N>(S, j, k, c);
  __syncthreads();
  const int i = a_idx;
  int z[N];
  read_row<N>(S, i, k, z);
  invN<KIND, N>(z);
  (void)store_row<N, DT, C::SROUND>(p.dst, w.pix0 + static_cast<int64_t>(i) * p.g.pitch + k * N,
                                    active, z, nullptr);
}

// ---------------------------------------------------------------- dispatch
template <int KIND, int N, int DT>
hipError_t launch_typed(Mode mode, const PassParams& p, hipStream_t s) {
  using C = Cfg<N>;
  const dim3 grid((p.g.tiles_x + C::TPW - 1) / C::TPW, p.g.tiles_y, p.g.batch);
  const bool quant = p.qstep > 0;
  switch (mode) {
    case Mode::Compress:
      if (quant) compress_jam<KIND, N, DT, true><<<grid, kBlock, 0, s>>>(p);
      else compress_jam<KIND, N, DT, false><<<grid, kBlock, 0, s>>>(p);
      break;
    case Mode::Forward:
      forward_jam<KIND, N, DT><<<grid, kBlock, 0, s>>>(p);
      break;
    case Mode::Inverse:
      if (quant) inverse_jam<KIND, N, DT, true, false><<<grid, kBlock, 0, s>>>(p);
      else inverse_jam<KIND, N, DT, false, false><<<grid, kBlock, 0, s>>>(p);
      break;
    case Mode::Decompress:
      if (quant) inverse_jam<KIND, N, DT, true, true><<<grid, kBlock, 0, s>>>(p);
      else inverse_jam<KIND, N, DT, false, true><<<grid, kBlock, 0, s>>>(p);
      break;
  }
  return hipGetLastError();
}

template <int KIND, int N>
hipError_t launch_n(Mode mode, int dtype, const PassParams& p, hipStream_t s) {
  return dtype == DT_U8 ? launch_typed<KIND, N, DT_U8>(mode, p, s)
                        : launch_typed<KIND, N, DT_I16>(mode, p, s);
}

}  // namespace

int launch_jam(Mode mode, int kind, int n, int dtype, const PassParams& p, hipStream_t stream) {
  if (kind == KIND_SIGN)
    return n == 16 ? launch_n<KIND_SIGN, 16>(mode, dtype, p, stream)
                   : launch_n<KIND_SIGN, 32>(mode, dtype, p, stream);
  return n == 16 ? launch_n<KIND_ROUND, 16>(mode, dtype, p, stream)
                 : launch_n<KIND_ROUND, 32>(mode, dtype, p, stream);
}

}  // namespace adct
