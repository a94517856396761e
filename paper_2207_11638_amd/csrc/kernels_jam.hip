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
#include "jam_group.hpp"

namespace adct {
namespace {

using namespace jam;

// ------------------------------------------------------------------ kernels
struct WgPos {
  int tx0, ty, img;
  int64_t tile0;   // global index of tile k = 0
  int64_t pix0;    // pixel offset of the top-left corner of tile k = 0
};

// Tile group gx (TPW tiles from tile column TPW gx) of tile row blockIdx.y of
// image blockIdx.z.
template <int N>
__device__ __forceinline__ WgPos wg_pos_at(const Geom& g, int gx, int ty, int img) {
  WgPos w;
  w.tx0 = gx * Cfg<N>::TPW;
  w.ty = ty;
  w.img = img;
  w.tile0 = (static_cast<int64_t>(w.img) * g.tiles_y + w.ty) * g.tiles_x + w.tx0;
  w.pix0 = static_cast<int64_t>(w.img) * g.image_stride +
           static_cast<int64_t>(w.ty) * N * g.pitch + static_cast<int64_t>(w.tx0) * N;
  return w;
}

template <int N>
__device__ __forceinline__ WgPos wg_pos(const Geom& g, int gx) {
  return wg_pos_at<N>(g, gx, blockIdx.y, blockIdx.z);
}

template <int N>
__device__ __forceinline__ GroupIO plain_io(const PassParams& p, const WgPos& w) {
  using C = Cfg<N>;
  const int k = threadIdx.x % C::TPW;
  GroupIO io;
  io.src = p.src;
  io.dst = p.dst;
  io.pitch = p.g.pitch;
  io.tile_pix = w.pix0 + static_cast<int64_t>(k) * N;
  io.nact = min(C::TPW, p.g.tiles_x - w.tx0);
  io.active = k < io.nact;
  io.r = p.r;
  io.kept = p.cout != nullptr ? p.cout + w.tile0 * p.r : nullptr;
  io.scaled = p.scaled != nullptr ? p.scaled + w.tile0 * p.r : nullptr;
  io.sse = p.sse != nullptr;
  return io;
}

// The workgroup walks p.gpw tile groups along its tile row and adds their
// error energy to the image's total with one atomic.  KB: compile-time bound
// on the kept rows and columns (zonal r <= KB (KB + 1) / 2), N otherwise.
template <int KIND, int N, int DT, bool QUANT, int KB>
__global__ __launch_bounds__(kBlock) void compress_jam(PassParams p) {
  using C = Cfg<N, kBlock, KB>;
  __shared__ int S[C::WORDS];
  __shared__ Shared<N> sh;
  __shared__ unsigned long long red[kBlock / 64];
  load_tables<KIND, N, kBlock, KB>(sh, p.t, p.r);
  const int img = blockIdx.z, ty = blockIdx.y, wx = blockIdx.x;
  const int groups_x = (p.g.tiles_x + C::TPW - 1) / C::TPW;
  const int g0 = wx * p.gpw;
  const int g1 = min(g0 + p.gpw, groups_x);
  unsigned long long e = 0;
  for (int gx = g0; gx < g1; ++gx)
    e += compress_group<KIND, N, DT, QUANT, kBlock, true, KB>(
        S, sh, plain_io<N>(p, wg_pos_at<N>(p.g, gx, ty, img)));
  if (p.sse != nullptr) block_add_sse<kBlock>(p.sse + img, e, red);
}

template <int KIND, int N, int DT>
__global__ __launch_bounds__(kBlock) void forward_jam(PassParams p) {
  using C = Cfg<N>;
  __shared__ int S[C::WORDS];
  const WgPos w = wg_pos<N>(p.g, blockIdx.x);
  const int a_idx = threadIdx.x / C::TPW;
  const int k = threadIdx.x % C::TPW;
  const GroupIO io = plain_io<N>(p, w);
  const int nact = io.nact;
  RowWords<N, DT> x;
  row_forward<KIND, N, DT, kBlock>(S, io, a_idx, k, x);
  __syncthreads();
  const int j = a_idx;
  int c[N];
  read_column<N, kBlock>(S, j, k, c);
  fwdN<KIND, N>(c);
  if constexpr (DT == DT_U8)
    if (j == 0) c[0] -= 128 * N * N;
  __syncthreads();
  write_column_rows<N, kBlock>(S, j, k, c);   // [k][v][u], row stride ZS
  __syncthreads();
  // natural order within a tile, tiles contiguous in global memory
  uint32_t* dst = reinterpret_cast<uint32_t*>(p.cout + w.tile0 * N * N);
  for (int e = threadIdx.x; e < nact * N * N; e += kBlock) {
    const int kk = e / (N * N), v = (e / N) % N, u = e % N;
    st_stream(dst + e, static_cast<uint32_t>(S[kk * C::TS + v * C::ZS + u]));
  }
}

// Inverse from natural-order coefficients (DECOMP = false) or from the
// zig-zag-ordered retained coefficients of adct_compress (DECOMP = true).
template <int KIND, int N, int DT, bool QUANT, bool DECOMP>
__global__ __launch_bounds__(kBlock) void inverse_jam(PassParams p) {
  using C = Cfg<N>;
  __shared__ int S[C::WORDS];
  __shared__ Shared<N> sh;
  const int r = p.r;
  load_tables<KIND, N, kBlock>(sh, p.t, r);
  const WgPos w = wg_pos<N>(p.g, blockIdx.x);
  const int a_idx = threadIdx.x / C::TPW;
  const int k = threadIdx.x % C::TPW;
  const bool active = w.tx0 + k < p.g.tiles_x;
  const int nact = min(C::TPW, p.g.tiles_x - w.tx0);
  __syncthreads();
  // stage this workgroup's coefficients (contiguous in global memory) into the
  // [k][v][u], row stride ZS layout; entries outside the zonal prefix are not read
  if constexpr (DECOMP) {
    const int32_t* src = p.cin + w.tile0 * r;
    if (threadIdx.x < nact * r) {
      int kk = threadIdx.x / r;
      int q = threadIdx.x - kk * r;
      const int dk = kBlock / r, dq = kBlock - dk * r;
      for (int e = threadIdx.x; e < nact * r; e += kBlock) {
        S[kk * C::TS + (zz_word<KIND, N>(sh, q) & 0xffff)] = src[e];
        q += dq;
        kk += dk;
        if (q >= r) {
          q -= r;
          ++kk;
        }
      }
    }
  } else {
    const int32_t* src = p.cin + w.tile0 * N * N;
    for (int e = threadIdx.x; e < nact * N * N; e += kBlock) {
      const int kk = e / (N * N), v = (e / N) % N, u = e % N;
      S[kk * C::TS + v * C::ZS + u] = src[e];
    }
  }
  __syncthreads();
  constexpr RowClasses<N> RC = row_classes<KIND, N>();
  const int j = a_idx;
  const int keep = active ? sh.cnt[j] : 0;
  const int cls_u = sh.cls[j];
  int c[N];
#pragma unroll
  for (int v = 0; v < N; ++v) {
    int b = S[k * C::TS + v * C::ZS + j];
    b = v < keep ? b : 0;
    if constexpr (QUANT) b = __mul24(b, sh.dq[RC.cls[v] * 4 + cls_u]);
    c[v] = b;
  }
  __syncthreads();
  invN<KIND, N>(c);
  if constexpr (QUANT) {
#pragma unroll
    for (int v = 0; v < N; ++v) c[v] >>= 1;
  }
  write_inverse_column<N, kBlock>(S, j, k, c);
  __syncthreads();
  const int i = a_idx;
  int z[N];
  read_row<N, kBlock>(S, i, k, z);
  invN<KIND, N>(z);
  (void)store_row<N, DT, C::SROUND>(p.dst, w.pix0 + static_cast<int64_t>(i) * p.g.pitch + k * N,
                                    active, z, nullptr);
}

// ---------------------------------------------------------------- dispatch
template <int KIND, int N, int DT>
hipError_t launch_typed(Mode mode, const PassParams& p_in, hipStream_t s) {
  using C = Cfg<N>;
  PassParams p = p_in;
  const int groups_x = (p.g.tiles_x + C::TPW - 1) / C::TPW;
  p.gpw = mode == Mode::Compress
              ? groups_per_wg(groups_x, static_cast<int64_t>(p.g.tiles_y) * p.g.batch)
              : 1;
  const dim3 grid((groups_x + p.gpw - 1) / p.gpw, p.g.tiles_y, p.g.batch);
  const bool quant = p.qstep > 0;
  switch (mode) {
    case Mode::Compress:
      // kept bound: r <= 10 keeps anti-diagonals 0..3, r <= 36 anti-diagonals 0..7
      if (quant) compress_jam<KIND, N, DT, true, N><<<grid, kBlock, 0, s>>>(p);
      else if (p.r <= 10) compress_jam<KIND, N, DT, false, 4><<<grid, kBlock, 0, s>>>(p);
      else if (p.r <= 36) compress_jam<KIND, N, DT, false, 8><<<grid, kBlock, 0, s>>>(p);
      else compress_jam<KIND, N, DT, false, N><<<grid, kBlock, 0, s>>>(p);
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

// 64-point level of the recursion: 8-bit input and zonal retention only (the
// int32 intermediates of its inverse are exact for 8-bit input, not over the
// whole int16 range); the host refuses the other cases.
template <int KIND>
hipError_t launch_64(Mode mode, const PassParams& p_in, hipStream_t s) {
  constexpr int N = 64;
  using C = Cfg<N>;
  PassParams p = p_in;
  const int groups_x = (p.g.tiles_x + C::TPW - 1) / C::TPW;
  p.gpw = mode == Mode::Compress
              ? groups_per_wg(groups_x, static_cast<int64_t>(p.g.tiles_y) * p.g.batch)
              : 1;
  const dim3 grid((groups_x + p.gpw - 1) / p.gpw, p.g.tiles_y, p.g.batch);
  switch (mode) {
    case Mode::Compress:
      if (p.r <= 10) compress_jam<KIND, N, DT_U8, false, 4><<<grid, kBlock, 0, s>>>(p);
      else if (p.r <= 36) compress_jam<KIND, N, DT_U8, false, 8><<<grid, kBlock, 0, s>>>(p);
      else compress_jam<KIND, N, DT_U8, false, N><<<grid, kBlock, 0, s>>>(p);
      break;
    case Mode::Forward:
      forward_jam<KIND, N, DT_U8><<<grid, kBlock, 0, s>>>(p);
      break;
    case Mode::Inverse:
      inverse_jam<KIND, N, DT_U8, false, false><<<grid, kBlock, 0, s>>>(p);
      break;
    case Mode::Decompress:
      inverse_jam<KIND, N, DT_U8, false, true><<<grid, kBlock, 0, s>>>(p);
      break;
  }
  return hipGetLastError();
}

}  // namespace

int launch_jam(Mode mode, int kind, int n, int dtype, const PassParams& p, hipStream_t stream) {
  if (n == 64)
    return kind == KIND_SIGN ? launch_64<KIND_SIGN>(mode, p, stream)
                             : launch_64<KIND_ROUND>(mode, p, stream);
  if (kind == KIND_SIGN)
    return n == 16 ? launch_n<KIND_SIGN, 16>(mode, dtype, p, stream)
                   : launch_n<KIND_SIGN, 32>(mode, dtype, p, stream);
  return n == 16 ? launch_n<KIND_ROUND, 16>(mode, dtype, p, stream)
                 : launch_n<KIND_ROUND, 32>(mode, dtype, p, stream);
}

}  // namespace adct
