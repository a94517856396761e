// 8 x 8 kernels: one thread owns one tile, one wave (= one workgroup) owns 64
// horizontally adjacent tiles of a tile row.
//
// A thread loads its 8 rows with one 8-byte (uint8) or 16-byte (int16) load
// per row, so each row load of the wave is one contiguous 512 B / 1 KB
// segment, and keeps the whole tile in registers.  Row and column
// butterflies, zonal masking or quantisation, the inverse butterflies and
// rounding all run in registers.  The per-tile coefficient outputs ([tile][r]
// words, r per thread) are staged through LDS so that every global store of
// the wave writes consecutive words: each thread first writes its r words at
// a row stride RS (odd, so the 64 concurrent LDS writes hit distinct banks),
// then the wave copies whole tiles with lane -> (tile, word) fixed per lane.
// The level shift of 8-bit input is folded into the DC coefficient: every AC
// row of T sums to zero, so T (A - 128) T^T differs from T A T^T only in
// b[0][0], by 128 N^2.
#include <algorithm>

#include "tile8.hpp"

namespace adct {
namespace {

using namespace t8;

// ------------------------------------------------------------------ kernels
// Fused forward -> retain/quantise -> inverse -> round -> store -> SSE.
// RB is a compile-time bound on r: zig-zag positions >= RB are known to be
// zero, so the compiler drops the arithmetic that only feeds or reads them.
// One wave covers 64 tiles (4096 pixels) and adds their error energy to the
// image's total with one atomic; the workgroups interleave p.spread images so
// that those atomics spread over several addresses.  (Walking several groups per
// wave, as the 16/32-point kernels do, makes the compiler keep the tables
// live across the loop and costs more registers than the atomics it saves.)
template <int KIND, int DT, int RB, bool QUANT>
__global__ __launch_bounds__(kWave) void compress8(PassParams p) {
  __shared__ int lds[kWave * row_stride(RB)];
  const WaveTiles w = wave_tiles_interleaved(p.g, p.spread);
  WaveIO io;
  io.src = p.src;
  io.dst = p.dst;
  io.pitch = p.g.pitch;
  io.tile_pix = w.pix;
  io.lane = w.lane;
  io.active = w.active;
  io.nact = w.nact;
  io.r = p.r;
  io.kept = p.cout != nullptr ? p.cout + w.tile0 * p.r : nullptr;
  io.scaled = p.scaled != nullptr ? p.scaled + w.tile0 * p.r : nullptr;
  io.sse = p.sse != nullptr;
  const unsigned long long e = compress_wave<KIND, DT, RB, QUANT, true>(lds, p.t, io);
  if (p.sse != nullptr) block_add_sse<kWave>(p.sse + w.img, e, nullptr);
}

template <int KIND, int DT>
__global__ __launch_bounds__(kWave) void forward8(PassParams p) {
  constexpr int RS = row_stride(kN * kN);
  __shared__ int lds[kWave * RS];
  const WaveTiles w = wave_tiles(p.g, blockIdx.x);
  Raw<DT> raw;
  load_raw<DT>(p.src, w.pix, p.g.pitch, w.active, raw);
  int a[kN][kN];
  unpack<DT>(raw, a);
  forward2d<KIND>(a);
  if constexpr (DT == DT_U8) a[0][0] -= 128 * kN * kN;
#pragma unroll
  for (int v = 0; v < kN; ++v)
#pragma unroll
    for (int u = 0; u < kN; ++u) lds[w.lane * RS + v * kN + u] = a[v][u];
  __syncthreads();
  // 16 lanes per tile, four words each: 16-byte stores of whole tiles
  const int lt = w.lane >> 4, gq = w.lane & 15;
  int4* out = reinterpret_cast<int4*>(p.cout + w.tile0 * kN * kN);
#pragma unroll
  for (int t0 = 0; t0 < kWave; t0 += 4) {
    const int t = t0 + lt;
    if (t < w.nact) {
      const int* s = lds + t * RS + 4 * gq;
      st_stream(reinterpret_cast<uint4*>(out + t * 16 + gq),
                make_uint4(s[0], s[1], s[2], s[3]));
    }
  }
}

// Inverse from natural-order coefficients (DECOMP = false) or from the
// zig-zag-ordered retained coefficients of adct_compress (DECOMP = true).
template <int KIND, int DT, bool QUANT, bool DECOMP>
__global__ __launch_bounds__(kWave) void inverse8(PassParams p) {
  constexpr int RS = row_stride(kN * kN);
  __shared__ int lds[kWave * RS];
  const WaveTiles w = wave_tiles(p.g, blockIdx.x);
  const int r = p.r;
  if constexpr (DECOMP) {
    const int32_t* g = p.cin + w.tile0 * r;
    if (r == kN * kN) copy_tiles_in<kN * kN>(lds, g, w.nact, w.lane);
    else copy_tiles_in_rt(lds, g, r, w.nact, w.lane);
  } else {
    const int lt = w.lane >> 4, gq = w.lane & 15;
    const int4* in = reinterpret_cast<const int4*>(p.cin + w.tile0 * kN * kN);
#pragma unroll
    for (int t0 = 0; t0 < kWave; t0 += 4) {
      const int t = t0 + lt;
      if (t < w.nact) {
        const int4 v = in[t * 16 + gq];
        int* s = lds + t * RS + 4 * gq;
        s[0] = v.x; s[1] = v.y; s[2] = v.z; s[3] = v.w;
      }
    }
  }
  __syncthreads();
  const int rs = DECOMP ? row_stride(r) : RS;
  int a[kN][kN];
#pragma unroll
  for (int v = 0; v < kN; ++v)
#pragma unroll
    for (int u = 0; u < kN; ++u) {
      const int pos = zz_pos(kN, v, u);
      int b = 0;
      if (w.active && pos < r) b = lds[w.lane * rs + (DECOMP ? pos : v * kN + u)];
      if constexpr (QUANT) b = __mul24(b, p.t.dq[table_index<KIND>(v, u)]);
      a[v][u] = b;
    }
  inverse2d<KIND>(a);
  constexpr int S = QUANT ? 9 : 8;
  Raw<DT> rec;
  round_pack<DT, S>(a, rec);
  if (w.active) store_raw<DT, true>(p.dst, w.pix, p.g.pitch, rec);
}

// ---------------------------------------------------------------- dispatch
constexpr int kRB[] = {1, 3, 6, 10, 15, 16, 21, 28, 36, 45, 64};
constexpr int kNumRB = sizeof(kRB) / sizeof(kRB[0]);

dim3 grid_for(const Geom& g) {
  return dim3((g.tiles_x + kWave - 1) / kWave, g.tiles_y, g.batch);
}

// The comparison transforms take a coarser set of bounds (fewer kernels to
// build); any bound >= r gives the same result.
constexpr bool coarse_rb(int rb) { return rb == 10 || rb == 28 || rb == 64; }

template <int KIND, int DT, int I>
void launch_compress_rb(const PassParams& p, hipStream_t s, dim3 grid) {
  if constexpr (I < kNumRB) {
    if constexpr (KIND <= KIND_ROUND || coarse_rb(kRB[I])) {
      if (p.r <= kRB[I]) {
        compress8<KIND, DT, kRB[I], false><<<grid, kWave, 0, s>>>(p);
        return;
      }
    }
    launch_compress_rb<KIND, DT, I + 1>(p, s, grid);
  }
}

template <int KIND, int DT>
hipError_t launch_typed(Mode mode, const PassParams& p_in, hipStream_t s) {
  PassParams p = p_in;
  p.gpw = 1;
  // images interleaved by the fused kernel: wide for small r, where the
  // per-workgroup error-energy atomics queue on one address, narrow for large
  // r, where the output stream wants raster order (measured per r on the C1
  // shape: 128 for r <= 10, 64 up to 16, 32 up to 28, 8 up to 45, 1 beyond)
  p.spread = std::min(p.g.batch,
                      p.r <= 10 ? 128 : (p.r <= 16 ? 64 : (p.r <= 28 ? 32 : (p.r <= 45 ? 8 : 1))));
  const dim3 grid = grid_for(p.g);
  const bool quant = p.qstep > 0;
  switch (mode) {
    case Mode::Compress:
      if (quant) compress8<KIND, DT, 64, true><<<grid, kWave, 0, s>>>(p);
      else launch_compress_rb<KIND, DT, 0>(p, s, grid);
      break;
    case Mode::Forward:
      forward8<KIND, DT><<<grid, kWave, 0, s>>>(p);
      break;
    case Mode::Inverse:
      if (quant) inverse8<KIND, DT, true, false><<<grid, kWave, 0, s>>>(p);
      else inverse8<KIND, DT, false, false><<<grid, kWave, 0, s>>>(p);
      break;
    case Mode::Decompress:
      if (quant) inverse8<KIND, DT, true, true><<<grid, kWave, 0, s>>>(p);
      else inverse8<KIND, DT, false, true><<<grid, kWave, 0, s>>>(p);
      break;
  }
  return hipGetLastError();
}

}  // namespace

int launch_n8(Mode mode, int kind, int dtype, const PassParams& p, hipStream_t stream) {
  if (kind == KIND_WHT)
    return dtype == DT_U8 ? launch_typed<KIND_WHT, DT_U8>(mode, p, stream)
                          : launch_typed<KIND_WHT, DT_I16>(mode, p, stream);
  if (kind == KIND_SDCT)
    return dtype == DT_U8 ? launch_typed<KIND_SDCT, DT_U8>(mode, p, stream)
                          : launch_typed<KIND_SDCT, DT_I16>(mode, p, stream);
  if (kind == KIND_HT)
    return dtype == DT_U8 ? launch_typed<KIND_HT, DT_U8>(mode, p, stream)
                          : launch_typed<KIND_HT, DT_I16>(mode, p, stream);
  if (kind == KIND_SIGN)
    return dtype == DT_U8 ? launch_typed<KIND_SIGN, DT_U8>(mode, p, stream)
                          : launch_typed<KIND_SIGN, DT_I16>(mode, p, stream);
  return dtype == DT_U8 ? launch_typed<KIND_ROUND, DT_U8>(mode, p, stream)
                        : launch_typed<KIND_ROUND, DT_I16>(mode, p, stream);
}

}  // namespace adct
