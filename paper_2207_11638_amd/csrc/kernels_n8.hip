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
#include "adct_internal.hpp"

namespace adct {
namespace {

constexpr int kN = 8;
constexpr int kWave = 64;

struct ZigZag8 {
  int v[64];
  int u[64];
};

constexpr ZigZag8 make_zigzag8() {
  ZigZag8 z{};
  for (int v = 0; v < kN; ++v)
    for (int u = 0; u < kN; ++u) {
      const int k = zz_pos(kN, v, u);
      z.v[k] = v;
      z.u[k] = u;
    }
  return z;
}

constexpr ZigZag8 kZZ = make_zigzag8();

constexpr int row_stride(int r) { return (r % 2) ? r : r + 1; }

// Packed pixel rows of one tile: uint8 -> 2 words per row, int16 -> 4.
template <int DT>
struct Raw {
  static constexpr int W = DT == DT_U8 ? 2 : 4;
  uint32_t w[kN][W];
};

// ---------------------------------------------------------------- pixel I/O
template <int DT>
__device__ __forceinline__ void load_raw(const void* src, int64_t off, int64_t pitch, bool active,
                                         Raw<DT>& raw) {
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    if constexpr (DT == DT_U8) {
      uint2 w = make_uint2(0x80808080u, 0x80808080u);
      if (active)
        w = *reinterpret_cast<const uint2*>(static_cast<const uint8_t*>(src) + off + i * pitch);
      raw.w[i][0] = w.x;
      raw.w[i][1] = w.y;
    } else {
      uint4 w = make_uint4(0u, 0u, 0u, 0u);
      if (active)
        w = *reinterpret_cast<const uint4*>(static_cast<const int16_t*>(src) + off + i * pitch);
      raw.w[i][0] = w.x;
      raw.w[i][1] = w.y;
      raw.w[i][2] = w.z;
      raw.w[i][3] = w.w;
    }
  }
}

template <int DT>
__device__ __forceinline__ void unpack(const Raw<DT>& raw, int (&a)[kN][kN]) {
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    if constexpr (DT == DT_U8) {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a[i][j] = (raw.w[i][0] >> (8 * j)) & 0xff;
        a[i][j + 4] = (raw.w[i][1] >> (8 * j)) & 0xff;
      }
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        a[i][2 * j] = static_cast<int>(raw.w[i][j] << 16) >> 16;
        a[i][2 * j + 1] = static_cast<int>(raw.w[i][j]) >> 16;
      }
    }
  }
}

// Round z / 2^S (half away from zero), shift/clip, pack.
template <int DT, int S>
__device__ __forceinline__ void round_pack(const int (&z)[kN][kN], Raw<DT>& out) {
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    int y[kN];
#pragma unroll
    for (int j = 0; j < kN; ++j) {
      if constexpr (DT == DT_U8)
        y[j] = round_shift_u8<S>(z[i][j]);
      else
        y[j] = min(max(round_shift<S>(z[i][j]), -32768), 32767);
    }
    if constexpr (DT == DT_U8) {
      out.w[i][0] = y[0] | (y[1] << 8) | (y[2] << 16) | (y[3] << 24);
      out.w[i][1] = y[4] | (y[5] << 8) | (y[6] << 16) | (y[7] << 24);
    } else {
#pragma unroll
      for (int j = 0; j < 4; ++j)
        out.w[i][j] = (y[2 * j] & 0xffff) | (static_cast<uint32_t>(y[2 * j + 1]) << 16);
    }
  }
}

template <int DT>
__device__ __forceinline__ void store_raw(void* dst, int64_t off, int64_t pitch, const Raw<DT>& raw) {
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    if constexpr (DT == DT_U8)
      st_stream(reinterpret_cast<uint2*>(static_cast<uint8_t*>(dst) + off + i * pitch),
                make_uint2(raw.w[i][0], raw.w[i][1]));
    else
      st_stream(reinterpret_cast<uint4*>(static_cast<int16_t*>(dst) + off + i * pitch),
                make_uint4(raw.w[i][0], raw.w[i][1], raw.w[i][2], raw.w[i][3]));
  }
}

// Sum of squared differences of two packed tiles.
template <int DT>
__device__ __forceinline__ unsigned long long tile_sse(const Raw<DT>& x, const Raw<DT>& y) {
  if constexpr (DT == DT_U8) {
    // sum (x - y)^2 = sum x^2 + sum y^2 - 2 sum x y, four bytes per dot step;
    // every partial sum of a tile stays below 2^23
    uint32_t sxx = 0, syy = 0, sxy = 0;
#pragma unroll
    for (int i = 0; i < kN; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        sxx = __builtin_amdgcn_udot4(x.w[i][j], x.w[i][j], sxx, false);
        syy = __builtin_amdgcn_udot4(y.w[i][j], y.w[i][j], syy, false);
        sxy = __builtin_amdgcn_udot4(x.w[i][j], y.w[i][j], sxy, false);
      }
    return sxx + syy - 2u * sxy;
  } else {
    unsigned long long e = 0;
#pragma unroll
    for (int i = 0; i < kN; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int d0 = (static_cast<int>(y.w[i][j] << 16) >> 16) - (static_cast<int>(x.w[i][j] << 16) >> 16);
        const int d1 = (static_cast<int>(y.w[i][j]) >> 16) - (static_cast<int>(x.w[i][j]) >> 16);
        e += static_cast<unsigned long long>(static_cast<long long>(d0) * d0) +
             static_cast<unsigned long long>(static_cast<long long>(d1) * d1);
      }
    return e;
  }
}

// ------------------------------------------------------------ 2D transforms
template <int KIND>
__device__ __forceinline__ void forward2d(int (&a)[kN][kN]) {
#pragma unroll
  for (int i = 0; i < kN; ++i) fwd8<KIND>(a[i]);          // rows:    A T^T
#pragma unroll
  for (int j = 0; j < kN; ++j) {                          // columns: T (A T^T)
    int c[kN];
#pragma unroll
    for (int i = 0; i < kN; ++i) c[i] = a[i][j];
    fwd8<KIND>(c);
#pragma unroll
    for (int i = 0; i < kN; ++i) a[i][j] = c[i];
  }
}

template <int KIND>
__device__ __forceinline__ void inverse2d(int (&a)[kN][kN]) {
#pragma unroll
  for (int j = 0; j < kN; ++j) {                          // columns: K B
    int c[kN];
#pragma unroll
    for (int i = 0; i < kN; ++i) c[i] = a[i][j];
    inv8<KIND>(c);
#pragma unroll
    for (int i = 0; i < kN; ++i) a[i][j] = c[i];
  }
#pragma unroll
  for (int i = 0; i < kN; ++i) inv8<KIND>(a[i]);          // rows:    (K B) K^T
}

__device__ __forceinline__ int quantise(int b, int32_t mq) {
  const uint32_t mag = static_cast<uint32_t>(b < 0 ? -b : b);
  const uint64_t prod = static_cast<uint64_t>(mag) * static_cast<uint32_t>(mq) + (1ull << 23);
  const int lev = static_cast<int>(prod >> 24);
  return b < 0 ? -lev : lev;
}

__device__ __forceinline__ int table_index(const Tables& t, int v, int u) {
  return t.cls[v] * 4 + t.cls[u];
}

__device__ __forceinline__ void add_sse(unsigned long long* sse, int img, unsigned long long e) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, kWave);
  if (threadIdx.x == 0 && e != 0) atomicAdd(sse + img, e);
}

struct WaveTiles {
  int lane, img, tx;
  int nact;        // active tiles of this wave (a prefix of the lanes)
  bool active;
  int64_t tile0;   // global index of the wave's first tile
  int64_t pix;     // pixel offset of this thread's tile
};

__device__ __forceinline__ WaveTiles wave_tiles(const Geom& g) {
  WaveTiles w;
  w.lane = threadIdx.x;
  const int tx0 = blockIdx.x * kWave;
  w.tx = tx0 + w.lane;
  w.img = blockIdx.z;
  w.nact = min(kWave, g.tiles_x - tx0);
  w.active = w.lane < w.nact;
  w.tile0 = (static_cast<int64_t>(w.img) * g.tiles_y + blockIdx.y) * g.tiles_x + tx0;
  w.pix = static_cast<int64_t>(w.img) * g.image_stride +
          static_cast<int64_t>(blockIdx.y) * kN * g.pitch + static_cast<int64_t>(w.tx) * kN;
  return w;
}

// ------------------------------------------------------ LDS staged tile words
// Copy the words staged at lds[t * RS + k] (t < nact, k < r) to g[t * r + k].
// Each pass covers q = 64 / r whole tiles; lane -> (tile lt, word kk) is fixed,
// so the addresses of every pass differ only by constants.
template <int R>
__device__ __forceinline__ void copy_tiles_out(uint32_t* g, const int* lds, int nact, int lane) {
  constexpr int RS = row_stride(R);
  constexpr int Q = kWave / R;
  const int lt = lane / R, kk = lane - (lane / R) * R;
  if (lane >= Q * R) return;
#pragma unroll
  for (int t0 = 0; t0 < kWave; t0 += Q) {
    const int t = t0 + lt;
    if (t < nact) {
      // a pass stores Q*R consecutive words: the streaming hint pays only when
      // that is a whole number of cache lines; otherwise L2 merges partial lines
      if constexpr (Q * R == kWave) st_stream(g + t * R + kk, static_cast<uint32_t>(lds[t * RS + kk]));
      else g[t * R + kk] = static_cast<uint32_t>(lds[t * RS + kk]);
    }
  }
}

__device__ __forceinline__ void copy_tiles_out_rt(uint32_t* g, const int* lds, int r, int rs,
                                                  int nact, int lane) {
  const int q = kWave / r;
  const int lt = lane / r, kk = lane - lt * r;
  if (lane >= q * r) return;
  for (int t = lt; t < nact; t += q) g[t * r + kk] = static_cast<uint32_t>(lds[t * rs + kk]);
}

// The reverse: g[t * r + k] -> lds[t * RS + k].
template <int R>
__device__ __forceinline__ void copy_tiles_in(int* lds, const int32_t* g, int nact, int lane) {
  constexpr int RS = row_stride(R);
  constexpr int Q = kWave / R;
  const int lt = lane / R, kk = lane - (lane / R) * R;
  if (lane >= Q * R) return;
#pragma unroll
  for (int t0 = 0; t0 < kWave; t0 += Q) {
    const int t = t0 + lt;
    if (t < nact) lds[t * RS + kk] = g[t * R + kk];
  }
}

__device__ __forceinline__ void copy_tiles_in_rt(int* lds, const int32_t* g, int r, int nact,
                                                 int lane) {
  const int rs = row_stride(r);
  const int q = kWave / r;
  const int lt = lane / r, kk = lane - lt * r;
  if (lane >= q * r) return;
  for (int t = lt; t < nact; t += q) lds[t * rs + kk] = g[t * r + kk];
}

// ------------------------------------------------------------------ kernels
// Fused forward -> retain/quantise -> inverse -> round -> store -> SSE.
// RB is a compile-time bound on r: zig-zag positions >= RB are known to be
// zero, so the compiler drops the arithmetic that only feeds or reads them.
template <int KIND, int DT, int RB, bool QUANT>
__global__ __launch_bounds__(kWave) void compress8(PassParams p) {
  constexpr int RS = row_stride(RB);
  __shared__ int lds[kWave * RS];
  const WaveTiles w = wave_tiles(p.g);
  Raw<DT> raw;
  load_raw<DT>(p.src, w.pix, p.g.pitch, w.active, raw);
  int a[kN][kN];
  unpack<DT>(raw, a);
  forward2d<KIND>(a);
  if constexpr (DT == DT_U8) a[0][0] -= 128 * kN * kN;

  const int r = p.r;
  // scaled coefficients s_v s_u b of the retained positions, in zig-zag order
  if (p.scaled != nullptr) {
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (k < r) {
        const int v = kZZ.v[k], u = kZZ.u[k];
        const float s = static_cast<float>(a[v][u]) * p.t.s2[table_index(p.t, v, u)];
        lds[w.lane * RS + k] = __builtin_bit_cast(int, s);
      }
    __syncthreads();
    uint32_t* g = reinterpret_cast<uint32_t*>(p.scaled + w.tile0 * r);
    if (r == RB) copy_tiles_out<RB>(g, lds, w.nact, w.lane);
    else copy_tiles_out_rt(g, lds, r, RS, w.nact, w.lane);
    __syncthreads();
  }
  // zonal mask (and quantisation) in place
#pragma unroll
  for (int v = 0; v < kN; ++v)
#pragma unroll
    for (int u = 0; u < kN; ++u) {
      const int pos = zz_pos(kN, v, u);
      if (pos >= RB) {
        a[v][u] = 0;
      } else {
        int b = pos < r ? a[v][u] : 0;
        if constexpr (QUANT) b = quantise(b, p.t.mq[table_index(p.t, v, u)]);
        a[v][u] = b;
      }
    }
  if (p.cout != nullptr) {
#pragma unroll
    for (int k = 0; k < RB; ++k)
      if (k < r) lds[w.lane * RS + k] = a[kZZ.v[k]][kZZ.u[k]];
    __syncthreads();
    uint32_t* g = reinterpret_cast<uint32_t*>(p.cout + w.tile0 * r);
    if (r == RB) copy_tiles_out<RB>(g, lds, w.nact, w.lane);
    else copy_tiles_out_rt(g, lds, r, RS, w.nact, w.lane);
  }
  if (p.dst == nullptr && p.sse == nullptr) return;
  if constexpr (QUANT) {
#pragma unroll
    for (int v = 0; v < kN; ++v)
#pragma unroll
      for (int u = 0; u < kN; ++u)
        if (zz_pos(kN, v, u) < RB) a[v][u] = __mul24(a[v][u], p.t.dq[table_index(p.t, v, u)]);
  }
  inverse2d<KIND>(a);
  // zonal: y = round(Z / (4 N^2)); quantised (one fractional bit): Z / (8 N^2)
  constexpr int S = QUANT ? 9 : 8;
  Raw<DT> rec;
  round_pack<DT, S>(a, rec);
  if (p.dst != nullptr && w.active) store_raw<DT>(p.dst, w.pix, p.g.pitch, rec);
  if (p.sse != nullptr) add_sse(p.sse, w.img, w.active ? tile_sse<DT>(raw, rec) : 0ull);
}

template <int KIND, int DT>
__global__ __launch_bounds__(kWave) void forward8(PassParams p) {
  constexpr int RS = row_stride(kN * kN);
  __shared__ int lds[kWave * RS];
  const WaveTiles w = wave_tiles(p.g);
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
  const WaveTiles w = wave_tiles(p.g);
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
      if constexpr (QUANT) b = __mul24(b, p.t.dq[table_index(p.t, v, u)]);
      a[v][u] = b;
    }
  inverse2d<KIND>(a);
  constexpr int S = QUANT ? 9 : 8;
  Raw<DT> rec;
  round_pack<DT, S>(a, rec);
  if (w.active) store_raw<DT>(p.dst, w.pix, p.g.pitch, rec);
}

// ---------------------------------------------------------------- dispatch
constexpr int kRB[] = {1, 3, 6, 10, 15, 16, 21, 28, 36, 45, 64};
constexpr int kNumRB = sizeof(kRB) / sizeof(kRB[0]);

dim3 grid_for(const Geom& g) {
  return dim3((g.tiles_x + kWave - 1) / kWave, g.tiles_y, g.batch);
}

template <int KIND, int DT, int I>
void launch_compress_rb(const PassParams& p, hipStream_t s, dim3 grid) {
  if constexpr (I < kNumRB) {
    if (p.r <= kRB[I]) {
      compress8<KIND, DT, kRB[I], false><<<grid, kWave, 0, s>>>(p);
      return;
    }
    launch_compress_rb<KIND, DT, I + 1>(p, s, grid);
  }
}

template <int KIND, int DT>
hipError_t launch_typed(Mode mode, const PassParams& p, hipStream_t s) {
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
  if (kind == KIND_SIGN)
    return dtype == DT_U8 ? launch_typed<KIND_SIGN, DT_U8>(mode, p, stream)
                          : launch_typed<KIND_SIGN, DT_I16>(mode, p, stream);
  return dtype == DT_U8 ? launch_typed<KIND_ROUND, DT_U8>(mode, p, stream)
                        : launch_typed<KIND_ROUND, DT_I16>(mode, p, stream);
}

}  // namespace adct
