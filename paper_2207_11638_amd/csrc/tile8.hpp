// Per-thread 8 x 8 tile processing, shared by the plain kernels and the
// ragged batch kernel.  One thread owns one tile; a wave owns up to 64 tiles.
#pragma once

#include "adct_internal.hpp"

namespace adct {
namespace t8 {

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
        w = ld_global(reinterpret_cast<const uint2*>(static_cast<const uint8_t*>(src) + off + i * pitch));
      raw.w[i][0] = w.x;
      raw.w[i][1] = w.y;
    } else {
      uint4 w = make_uint4(0u, 0u, 0u, 0u);
      if (active)
        w = ld_global(reinterpret_cast<const uint4*>(static_cast<const int16_t*>(src) + off + i * pitch));
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

template <int DT, bool NT>
__device__ __forceinline__ void store_raw(void* dst, int64_t off, int64_t pitch, const Raw<DT>& raw) {
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    if constexpr (DT == DT_U8)
      st_pix<NT>(reinterpret_cast<uint2*>(static_cast<uint8_t*>(dst) + off + i * pitch),
                make_uint2(raw.w[i][0], raw.w[i][1]));
    else
      st_pix<NT>(reinterpret_cast<uint4*>(static_cast<int16_t*>(dst) + off + i * pitch),
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

__device__ __forceinline__ int quantise(int b, int32_t mq) { return quantise_level(b, quant_mult(mq)); }

// Index of (v, u) in the class tables; the row classes of T8 are known at
// compile time, so with unrolled v, u this folds to a constant offset.
template <int KIND>
__device__ __forceinline__ int table_index(int v, int u) {
  constexpr RowClasses<kN> rc = row_classes<KIND, kN>();
  return rc.cls[v] * 4 + rc.cls[u];
}

// Where this thread's tile lives and where its wave's outputs go.
struct WaveIO {
  const void* src;
  void* dst;                  // reconstruction base (nullable)
  int64_t pitch;              // pixels
  int64_t tile_pix;           // pixel offset of this thread's tile
  int lane;                   // 0..63
  bool active;                // this thread's tile exists
  int nact;                   // tiles of the wave (lanes < nact are active)
  int r;                      // retained coefficients per tile
  int32_t* kept;              // [nact][r] block of this wave (nullable)
  float* scaled;              // [nact][r] block of this wave (nullable)
  bool sse;                   // compute the error energy
};

struct WaveTiles {
  int lane, img, tx;
  int nact;        // active tiles of this wave (a prefix of the lanes)
  bool active;
  int64_t tile0;   // global index of the wave's first tile
  int64_t pix;     // pixel offset of this thread's tile
};

// Tiles of group gx (64 tiles from tile column 64 gx) of tile row ty of
// image img.
__device__ __forceinline__ WaveTiles wave_tiles_at(const Geom& g, int gx, int ty, int img) {
  WaveTiles w;
  w.lane = threadIdx.x;
  const int tx0 = gx * kWave;
  w.tx = tx0 + w.lane;
  w.img = img;
  w.nact = min(kWave, g.tiles_x - tx0);
  w.active = w.lane < w.nact;
  w.tile0 = (static_cast<int64_t>(w.img) * g.tiles_y + ty) * g.tiles_x + tx0;
  w.pix = static_cast<int64_t>(w.img) * g.image_stride +
          static_cast<int64_t>(ty) * kN * g.pitch + static_cast<int64_t>(w.tx) * kN;
  return w;
}

// Tiles of group gx of tile row blockIdx.y of image blockIdx.z.
__device__ __forceinline__ WaveTiles wave_tiles(const Geom& g, int gx) {
  return wave_tiles_at(g, gx, blockIdx.y, blockIdx.z);
}

// The same tiles with the images interleaved s at a time: the linear
// workgroup index l of a (groups_x, tiles_y, batch) grid walks the images in
// blocks of s (the last block holds batch mod s), and inside a block takes
// image fastest, then group, then tile row; a bijection of the grid.  The
// workgroups resident at one time then belong to s images, so the one
// error-energy atomic per workgroup spreads over s addresses, while the
// workgroups that share a row of an image stay close in dispatch order
// (their row segments share DRAM pages).  The host picks s: wide where the
// atomics dominate (small r), narrow where the output stream does.  It
// keeps every grid below 2^32 workgroups, so 32-bit arithmetic suffices.
__device__ __forceinline__ WaveTiles wave_tiles_interleaved(const Geom& g, int s) {
  const uint32_t l = blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z);
  const uint32_t gxn = gridDim.x;
  const uint32_t per_image = gxn * static_cast<uint32_t>(g.tiles_y);
  const uint32_t S = static_cast<uint32_t>(s);
  const uint32_t full = static_cast<uint32_t>(g.batch) / S;
  uint32_t blk, within, width;
  if (l < full * S * per_image) {
    blk = l / (S * per_image);
    within = l - blk * S * per_image;
    width = S;
  } else {
    blk = full;
    within = l - full * S * per_image;
    width = static_cast<uint32_t>(g.batch) - full * S;
  }
  const uint32_t q = within / width;
  const int img = static_cast<int>(blk * S + (within - q * width));
  const uint32_t ty = q / gxn;
  return wave_tiles_at(g, static_cast<int>(q - ty * gxn), static_cast<int>(ty), img);
}

// ------------------------------------------------------ LDS staged tile words
// Copy the words staged at lds[t * RS + k] (t < nact, k < r) to g[t * r + k].
// Pass p stores words 64 p .. 64 p + 63 of the wave's [nact][r] block, one per
// lane: every pass writes 64 consecutive words, which are two whole 128-byte
// lines when the block starts on a 256-byte boundary (the plain kernels: a
// wave's block starts at tile 64 w); NT then selects the streaming hint.
// When r divides 64 the lane -> (tile, word) map is the same in every pass
// and the addresses differ only by constants; otherwise the tile and word of
// each lane step by (64 / r, 64 mod r).
template <int R, bool NT>
__device__ __forceinline__ void copy_tiles_out(uint32_t* g, const int* lds, int nact, int lane) {
  constexpr int RS = row_stride(R);
  constexpr int Q = kWave / R;
  if constexpr (Q * R == kWave) {
    const int lt = lane / R, kk = lane - (lane / R) * R;
#pragma unroll
    for (int t0 = 0; t0 < kWave; t0 += Q) {
      const int t = t0 + lt;
      if (t < nact) st_pix<NT>(g + t * R + kk, static_cast<uint32_t>(lds[t * RS + kk]));
    }
  } else {
    const int total = nact * R;
#pragma unroll
    for (int pass = 0; pass < R; ++pass) {   // 64 tiles x R words / 64 lanes
      const int e = pass * kWave + lane;
      if (e < total) {
        const int t = e / R, k = e - (e / R) * R;
        st_pix<NT>(g + e, static_cast<uint32_t>(lds[t * RS + k]));
      }
    }
  }
}

template <bool NT>
__device__ __forceinline__ void copy_tiles_out_rt(uint32_t* g, const int* lds, int r, int rs,
                                                  int nact, int lane) {
  const int total = nact * r;
  if (lane >= total) return;
  int t = lane / r, k = lane - (lane / r) * r;
  const int dt = kWave / r, dk = kWave - dt * r;
  for (int e = lane; e < total; e += kWave) {
    st_pix<NT>(g + e, static_cast<uint32_t>(lds[t * rs + k]));
    t += dt;
    k += dk;
    if (k >= r) {
      k -= r;
      ++t;
    }
  }
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


// ------------------------------------------------------------- fused wave
// Forward -> retain/quantise -> (outputs) -> inverse -> round -> store of the
// wave's tiles; returns this thread's squared reconstruction error (0 unless
// io.sse is set and the tile exists).  RB is a compile-time bound on r:
// zig-zag positions >= RB are known to be zero, so the compiler drops the
// arithmetic that only feeds or reads them.  With STAGED the [tile][r]
// outputs go through ``lds`` (64 * row_stride(RB) words owned by this wave)
// for coalesced stores; otherwise each thread stores its own r words.  Every
// thread of the workgroup must call this (it synchronises with
// __syncthreads when STAGED).  NT selects non-temporal reconstruction stores.
// TAB is the type of the constant tables (a Tables in kernel-argument or
// constant memory, read with scalar loads).
template <int KIND, int DT, int RB, bool QUANT, bool STAGED, bool NT = true, typename TAB>
__device__ __forceinline__ unsigned long long compress_wave(int* lds, const TAB& t, const WaveIO& io) {
  constexpr int RS = row_stride(RB);
  Raw<DT> raw;
  load_raw<DT>(io.src, io.tile_pix, io.pitch, io.active, raw);
  int a[kN][kN];
  unpack<DT>(raw, a);
  forward2d<KIND>(a);
  if constexpr (DT == DT_U8) a[0][0] -= 128 * kN * kN;

  const int r = io.r;
  const int lane = io.lane;
  // scaled coefficients s_v s_u b of the retained positions, in zig-zag order
  if (io.scaled != nullptr) {
    if constexpr (STAGED) {
#pragma unroll
      for (int k = 0; k < RB; ++k)
        if (k < r) {
          const int v = kZZ.v[k], u = kZZ.u[k];
          const float s = static_cast<float>(a[v][u]) * t.s2[table_index<KIND>(v, u)];
          lds[lane * RS + k] = __builtin_bit_cast(int, s);
        }
      __syncthreads();
      uint32_t* g = reinterpret_cast<uint32_t*>(io.scaled);
      if (r == RB) copy_tiles_out<RB, NT>(g, lds, io.nact, lane);
      else copy_tiles_out_rt<NT>(g, lds, r, RS, io.nact, lane);
      __syncthreads();
    } else if (io.active) {
#pragma unroll
      for (int k = 0; k < RB; ++k)
        if (k < r) {
          const int v = kZZ.v[k], u = kZZ.u[k];
          io.scaled[lane * r + k] = static_cast<float>(a[v][u]) * t.s2[table_index<KIND>(v, u)];
        }
    }
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
        if constexpr (QUANT) b = quantise(b, t.mq[table_index<KIND>(v, u)]);
        a[v][u] = b;
      }
    }
  if (io.kept != nullptr) {
    if constexpr (STAGED) {
#pragma unroll
      for (int k = 0; k < RB; ++k)
        if (k < r) lds[lane * RS + k] = a[kZZ.v[k]][kZZ.u[k]];
      __syncthreads();
      uint32_t* g = reinterpret_cast<uint32_t*>(io.kept);
      if (r == RB) copy_tiles_out<RB, NT>(g, lds, io.nact, lane);
      else copy_tiles_out_rt<NT>(g, lds, r, RS, io.nact, lane);
      __syncthreads();
    } else if (io.active) {
#pragma unroll
      for (int k = 0; k < RB; ++k)
        if (k < r) io.kept[lane * r + k] = a[kZZ.v[k]][kZZ.u[k]];
    }
  }
  if (io.dst == nullptr && !io.sse) return 0ull;
  if constexpr (QUANT) {
#pragma unroll
    for (int v = 0; v < kN; ++v)
#pragma unroll
      for (int u = 0; u < kN; ++u)
        if (zz_pos(kN, v, u) < RB) a[v][u] = __mul24(a[v][u], t.dq[table_index<KIND>(v, u)]);
  }
  inverse2d<KIND>(a);
  // zonal: y = round(Z / (4 N^2)); quantised (one fractional bit): Z / (8 N^2)
  constexpr int S = QUANT ? 9 : 8;
  Raw<DT> rec;
  round_pack<DT, S>(a, rec);
  if (io.dst != nullptr && io.active) store_raw<DT, NT>(io.dst, io.tile_pix, io.pitch, rec);
  return io.sse && io.active ? tile_sse<DT>(raw, rec) : 0ull;
}

}  // namespace t8
}  // namespace adct
