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
  io.sse = p.sse != nullptr ? p.sse + w.img : nullptr;
  return io;
}

template <int KIND, int N, int DT, bool QUANT>
__global__ __launch_bounds__(kBlock) void compress_jam(PassParams p) {
  using C = Cfg<N>;
  __shared__ int S[C::WORDS];
  __shared__ Shared sh;
  load_tables(sh, p.t, N);
  const WgPos w = wg_pos<N>(p.g);
  compress_group<KIND, N, DT, QUANT>(S, sh, plain_io<N>(p, w));
}

template <int KIND, int N, int DT>
__global__ __launch_bounds__(kBlock) void forward_jam(PassParams p) {
  using C = Cfg<N>;
  __shared__ int S[C::WORDS];
  const WgPos w = wg_pos<N>(p.g);
  const int a_idx = threadIdx.x / C::TPW;
  const int k = threadIdx.x % C::TPW;
  const GroupIO io = plain_io<N>(p, w);
  const int nact = io.nact;
  int x[N];
  row_forward<KIND, N, DT, kBlock>(S, io, a_idx, k, x);
  __syncthreads();
  const int j = a_idx;
  int c[N];
  read_column<N, kBlock>(S, j, k, c);
  fwdN<KIND, N>(c);
  if constexpr (DT == DT_U8)
    if (j == 0) c[0] -= 128 * N * N;
  __syncthreads();
  // natural order within a tile, tiles contiguous: dense staging [k][v][u]
#pragma unroll
  for (int v = 0; v < N; ++v) S[k * N * N + v * N + j] = c[v];
  __syncthreads();
  copy_out<kBlock>(reinterpret_cast<uint32_t*>(p.cout + w.tile0 * N * N), S, nact * N * N);
}

// Inverse from natural-order coefficients (DECOMP = false) or from the
// zig-zag-ordered retained coefficients of adct_compress (DECOMP = true).
template <int KIND, int N, int DT, bool QUANT, bool DECOMP>
__global__ __launch_bounds__(kBlock) void inverse_jam(PassParams p) {
  using C = Cfg<N>;
  __shared__ int S[C::WORDS];
  __shared__ Shared sh;
  load_tables(sh, p.t, N);
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
  write_column_rows<N, kBlock>(S, j, k, c);
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
