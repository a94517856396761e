// Workgroup-level processing of 16 x 16 and 32 x 32 tiles (Chen-JAM
// transforms of section 6.1), shared by the plain kernels and the ragged
// batch kernel; the same code also runs 8 x 8 tiles (eqs. 4, 5 and 6, 7) in
// the ragged batch, one thread per tile row.
//
// A workgroup of 256 threads owns TPW = 256/N tiles k = 0..TPW-1, each at its
// own pixel offset.  Thread L plays two roles:
//   row role    (i = L / TPW, k = L % TPW): row i of tile k;
//   column role (j = L / TPW, k = L % TPW): column j of tile k.
// When the tiles are horizontally adjacent (plain kernels) the lanes of a
// wave cover whole tile rows, so every pixel load/store of a wave is a run of
// 256 B (uint8) or 512 B (int16) per image row.  Each 1D N-point butterfly
// runs on N values in one thread's registers; the row<->column exchange goes
// through LDS with a padded layout (column stride N+1, tile stride 32/TPW mod
// 32 words) that keeps the LDS accesses of a half-wave on few banks.  The
// coefficients that leave in zig-zag order sit in a [v][u] layout of row
// stride ZS = N+2 (N+1 for N = 8).  Consecutive zig-zag positions step along
// anti-diagonals, (v, u) -> (v+1, u-1), which moves ZS - 1 words: at ZS = N+1
// that is N words, a multiple of the 32 banks for N = 32 and 64, and the
// lanes of one gather read that share an anti-diagonal (up to 26 of 32 at
// N = 32) queue on one bank; at N+2 a step moves N+1 words and at most 4 of
// 32 lanes meet on a bank.
//
// The kept bound KB (every retained coefficient has v, u < KB) also bounds
// what crosses LDS: KB transformed columns after the row pass, KB coefficient
// rows after the column pass and KB inverse columns before the last pass.
// A tile then needs max(KB (N+1), N (KB+1), KB ZS) words instead of N ZS.
#pragma once

#include "adct_internal.hpp"

namespace adct {
namespace jam {

// Smallest tile stride >= `words` that is congruent to `spread` modulo 32:
// the TPW tiles of a half-wave then start on banks `spread` apart.
constexpr int tile_stride(int words, int spread) {
  int ts = words;
  while (ts % 32 != spread) ++ts;
  return ts;
}

// With 32 tiles per workgroup (N = 8) any odd stride puts the 32 tiles of a
// half-wave on 32 distinct banks.
constexpr int odd_stride(int words) { return words | 1; }

// Row stride of the [v][u] coefficient layout (see the header comment).
constexpr int coef_stride(int n) { return n == 8 ? n + 1 : n + 2; }

template <int N, int BS = 256, int KB = N>
struct Cfg {
  static constexpr int TPW = BS / N;                        // tiles per workgroup
  static constexpr int CS = N + 1;                          // column stride of the forward exchange
  static constexpr int IS = KB + 1;                         // row stride of the inverse exchange
  static constexpr int ZS = coef_stride(N);                 // row stride of the coefficients
  static constexpr int NEED0 = KB * CS > N * IS ? KB * CS : N * IS;
  static constexpr int NEED = NEED0 > KB * ZS ? NEED0 : KB * ZS;
  static constexpr int TS = TPW == 32 ? odd_stride(NEED)   // LDS tile stride (words)
                                       : tile_stride(NEED, 32 / TPW);
  static constexpr int WORDS = TPW * TS;
  static constexpr int LOG2N = N == 8 ? 3 : (N == 16 ? 4 : (N == 32 ? 5 : 6));
  static constexpr int SROUND = 2 + 2 * LOG2N;              // divide by 4 N^2
  static_assert(TPW >= 2 && TPW <= 32, "unsupported block size");
  static_assert(KB == 4 || KB == 8 || KB == N, "unsupported kept bound");
};

constexpr int kBlock = 256;
constexpr int kMaxWords = Cfg<32>::WORDS;

// The zig-zag table is staged in LDS for N <= 32.  At N = 64 it would take
// 16 KB of the workgroup's 84 KB and hold the full-bound launch to one
// workgroup per compute unit; there it is read from constant memory.
template <int N>
constexpr bool zz_in_lds() { return N <= 32; }

// Constant tables of one (transform, N, qstep, r), staged in LDS.
//   zz[p]  (p < r): zig-zag position p of a tile, as its word offset
//          v ZS + u in the [v][u] coefficient layout (low 16 bits) and its
//          class-table entry cls[v] * 4 + cls[u] (high bits) (N <= 32);
//   cnt[u]: rows kept in column u (the zig-zag prefix keeps rows 0..cnt-1).
template <int N>
struct Shared {
  int32_t mq[16];
  int32_t dq[16];
  float s2[16];
  int32_t cls[N];
  int32_t cnt[N];
  int32_t zz[zz_in_lds<N>() ? N * N : 1];
};

// Zig-zag words of one (transform, N): entry p holds the word offset
// v ZS + u, in the [v][u] coefficient layout, of the coefficient at scan
// position p (low 16 bits) and its class-table entry cls[v] * 4 + cls[u]
// (high bits).  Built at compile time from the row classes of the forward
// butterfly, the numbering the host tables use.
template <int N>
struct ZigzagWords {
  int32_t w[N * N];
};

template <int KIND, int N>
constexpr ZigzagWords<N> make_zigzag_words() {
  const RowClasses<N> rc = row_classes<KIND, N>();
  ZigzagWords<N> z{};
  for (int v = 0; v < N; ++v)
    for (int u = 0; u < N; ++u)
      z.w[zz_pos(N, v, u)] = (v * coef_stride(N) + u) | ((rc.cls[v] * 4 + rc.cls[u]) << 16);
  return z;
}

template <int KIND, int N>
static __constant__ ZigzagWords<N> kZigzagWords = make_zigzag_words<KIND, N>();

// Zig-zag word p of a group's tables: from LDS, or from constant memory at
// N = 64.
template <int KIND, int N>
__device__ __forceinline__ int zz_word(const Shared<N>& sh, int p) {
  if constexpr (zz_in_lds<N>()) return sh.zz[p];
  else return kZigzagWords<KIND, N>.w[p];
}

// Kept rows of column u < 8 when the first r <= 64 zig-zag positions of an
// 8 x 8 block are retained (the zig-zag prefix keeps rows 0 .. c[r][u] - 1).
// The first eight anti-diagonals (positions below 36) are scanned in the
// same order for every N >= 8, so for r <= 36 the same counts hold for the
// first eight columns of any N x N block.
struct KeepRows8 {
  uint8_t c[65][8];
};

constexpr KeepRows8 make_keep_rows8() {
  KeepRows8 k{};
  for (int r = 0; r <= 64; ++r)
    for (int u = 0; u < 8; ++u) {
      int c = 0;
      while (c < 8 && zz_pos(8, c, u) < r) ++c;
      k.c[r][u] = static_cast<uint8_t>(c);
    }
  return k;
}

static __constant__ KeepRows8 kKeepRows8 = make_keep_rows8();

// Whether a group of N x N tiles with kept bound KB reads its kept-row counts
// from kKeepRows8 (8 x 8 tiles, or a bound of 4 or 8 columns: r <= 36) rather
// than from the workgroup's tables.
template <int N, int KB>
constexpr bool keep_from_table() {
  return N == 8 || KB < N;
}

// Fill the tables of one workgroup.  Thread p < r copies zig-zag word p;
// where the kept-row counts are needed from LDS (keep_from_table false),
// thread u < N counts the kept rows of column u by binary lifting (zz_pos(N,
// v, u) grows with v, so the kept rows are a prefix).  The tables depend on
// r and on the row classes of `t` only, not on LDS, so no barrier is needed
// before this.  The caller synchronises before the first use.
template <int KIND, int N, int BS, int KB = N>
__device__ __forceinline__ void load_tables(Shared<N>& sh, const Tables& t, int r) {
  const int i = threadIdx.x;
  if (i < 16) {
    sh.mq[i] = t.mq[i];
    sh.dq[i] = t.dq[i];
    sh.s2[i] = t.s2[i];
  }
  if (i < N) {
    sh.cls[i] = t.cls[i];
    if constexpr (!keep_from_table<N, KB>()) {
      int cnt = 0;   // largest cnt with zz_pos(N, cnt - 1, i) < r, by binary lifting
#pragma unroll
      for (int step = N; step > 0; step >>= 1)
        if (cnt + step <= N && zz_pos(N, cnt + step - 1, i) < r) cnt += step;
      sh.cnt[i] = cnt;
    }
  }
  if constexpr (zz_in_lds<N>()) {
#pragma unroll
    for (int q = 0; q < (N * N + BS - 1) / BS; ++q) {
      const int p = i + q * BS;
      if (p < r) sh.zz[p] = kZigzagWords<KIND, N>.w[p];
    }
  }
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
  bool sse;                   // compute the error energy
};

// ------------------------------------------------------------- pixel rows
// One row of one tile as loaded: N/4 words of packed uint8 or N/2 words of
// packed int16.  The words stay live until the reconstruction is compared
// with them, which for 8-bit pixels takes three dot-product steps per four
// pixels.
template <int N, int DT>
struct RowWords {
  static constexpr int W = DT == DT_U8 ? N / 4 : N / 2;
  uint32_t w[W];
};

template <int N, int DT>
__device__ __forceinline__ void load_row(const void* src, int64_t off, bool active,
                                         RowWords<N, DT>& rw) {
  constexpr int V = RowWords<N, DT>::W / 4;  // uint4 per row
  const uint32_t fill = DT == DT_U8 ? 0x80808080u : 0u;
  if constexpr (RowWords<N, DT>::W == 2) {   // 8 uint8 pixels
    uint2 w = make_uint2(fill, fill);
    if (active)
      w = ld_global(reinterpret_cast<const uint2*>(static_cast<const uint8_t*>(src) + off));
    rw.w[0] = w.x;
    rw.w[1] = w.y;
    return;
  }
  const uint4* p = reinterpret_cast<const uint4*>(static_cast<const uint8_t*>(src) +
                                                  off * (DT == DT_U8 ? 1 : 2));
#pragma unroll
  for (int q = 0; q < V; ++q) {
    uint4 w = make_uint4(fill, fill, fill, fill);
    if (active) w = ld_global(p + q);
    rw.w[4 * q] = w.x;
    rw.w[4 * q + 1] = w.y;
    rw.w[4 * q + 2] = w.z;
    rw.w[4 * q + 3] = w.w;
  }
}

template <int N, int DT>
__device__ __forceinline__ void unpack_row(const RowWords<N, DT>& rw, int (&x)[N]) {
  if constexpr (DT == DT_U8) {
#pragma unroll
    for (int d = 0; d < N / 4; ++d)
#pragma unroll
      for (int b = 0; b < 4; ++b) x[4 * d + b] = (rw.w[d] >> (8 * b)) & 0xff;
  } else {
#pragma unroll
    for (int d = 0; d < N / 2; ++d) {
      x[2 * d] = static_cast<int>(rw.w[d] << 16) >> 16;
      x[2 * d + 1] = static_cast<int>(rw.w[d]) >> 16;
    }
  }
}

// Round z / 2^S half away from zero, clip, store one row; return its squared
// error against the row as loaded (when x is given).
template <int N, int DT, int S, bool NT = true>
__device__ __forceinline__ unsigned long long store_row(void* dst, int64_t off, bool active,
                                                        const int (&z)[N],
                                                        const RowWords<N, DT>* x) {
  RowWords<N, DT> yw;
  if constexpr (DT == DT_U8) {
#pragma unroll
    for (int d = 0; d < N / 4; ++d)
      yw.w[d] = pack_round_u8<S>(z[4 * d], z[4 * d + 1], z[4 * d + 2], z[4 * d + 3]);
  } else {
#pragma unroll
    for (int d = 0; d < N / 2; ++d) {
      const int y0 = min(max(round_shift<S>(z[2 * d]), -32768), 32767);
      const int y1 = min(max(round_shift<S>(z[2 * d + 1]), -32768), 32767);
      yw.w[d] = (static_cast<uint32_t>(y0) & 0xffffu) | (static_cast<uint32_t>(y1) << 16);
    }
  }
  unsigned long long err = 0;
  if (x != nullptr) {
    if constexpr (DT == DT_U8) {
      // sum (x - y)^2 = sum x^2 + sum y^2 - 2 sum x y; a row's partial sums
      // stay below 2^21
      uint32_t sxx = 0, syy = 0, sxy = 0;
#pragma unroll
      for (int d = 0; d < N / 4; ++d) {
        sxx = __builtin_amdgcn_udot4(x->w[d], x->w[d], sxx, false);
        syy = __builtin_amdgcn_udot4(yw.w[d], yw.w[d], syy, false);
        sxy = __builtin_amdgcn_udot4(x->w[d], yw.w[d], sxy, false);
      }
      err = sxx + syy - 2u * sxy;
    } else {
#pragma unroll
      for (int d = 0; d < N / 2; ++d) {
        const long long d0 = (static_cast<int>(yw.w[d] << 16) >> 16) -
                             (static_cast<int>(x->w[d] << 16) >> 16);
        const long long d1 = (static_cast<int>(yw.w[d]) >> 16) - (static_cast<int>(x->w[d]) >> 16);
        err += static_cast<unsigned long long>(d0 * d0 + d1 * d1);
      }
    }
  }
  if (dst != nullptr && active) {
    if constexpr (RowWords<N, DT>::W == 2) {   // 8 uint8 pixels
      st_pix<NT>(reinterpret_cast<uint2*>(static_cast<uint8_t*>(dst) + off),
                 make_uint2(yw.w[0], yw.w[1]));
      return err;
    }
    uint4* p = reinterpret_cast<uint4*>(static_cast<uint8_t*>(dst) + off * (DT == DT_U8 ? 1 : 2));
#pragma unroll
    for (int q = 0; q < RowWords<N, DT>::W / 4; ++q)
      st_pix<NT>(p + q, make_uint4(yw.w[4 * q], yw.w[4 * q + 1], yw.w[4 * q + 2], yw.w[4 * q + 3]));
  }
  return err;
}

__device__ __forceinline__ int quantise(int b, int32_t mq) { return quantise_level(b, quant_mult(mq)); }

// Column j of tile k after the row pass (stored column-major, j < KB).
template <int N, int BS, int KB = N>
__device__ __forceinline__ void read_column(const int* S, int j, int k, int (&c)[N]) {
  using C = Cfg<N, BS, KB>;
#pragma unroll
  for (int v = 0; v < N; ++v) c[v] = S[k * C::TS + j * C::CS + v];
}

// Rows v < ROWS of column j into the coefficient layout [k][v][u] (row stride
// ZS, the layout the zig-zag table addresses).
template <int N, int BS, int ROWS = N, int KB = N>
__device__ __forceinline__ void write_column_rows(int* S, int j, int k, const int (&c)[N]) {
  using C = Cfg<N, BS, KB>;
#pragma unroll
  for (int v = 0; v < ROWS; ++v) S[k * C::TS + v * C::ZS + j] = c[v];
}

// Inverse exchange: column j < KB of tile k after the inverse column pass,
// stored row-major with row stride KB + 1.
template <int N, int BS, int KB = N>
__device__ __forceinline__ void write_inverse_column(int* S, int j, int k, const int (&c)[N]) {
  using C = Cfg<N, BS, KB>;
#pragma unroll
  for (int v = 0; v < N; ++v) S[k * C::TS + v * C::IS + j] = c[v];
}

// Row i of tile k from the inverse exchange; entries u >= KB are zero and
// not read.
template <int N, int BS, int KB = N>
__device__ __forceinline__ void read_row(const int* S, int i, int k, int (&z)[N]) {
  using C = Cfg<N, BS, KB>;
#pragma unroll
  for (int u = 0; u < N; ++u) z[u] = u < KB ? S[k * C::TS + i * C::IS + u] : 0;
}

// Copy ``count`` contiguous words from LDS to global memory (all threads).
template <int BS>
__device__ __forceinline__ void copy_out(uint32_t* dst, const int* src, int count) {
  for (int e = threadIdx.x; e < count; e += BS) st_stream(dst + e, static_cast<uint32_t>(src[e]));
}

// Zig-zag outputs of the group: element e = k r + p of the [nact][r] block is
// coefficient p (zig-zag order) of tile k, read from the [k][v][u]
// coefficient layout in S.  Kept values are the coefficients themselves
// (zonal) or their quantisation levels; scaled values are the coefficients
// times 1/sqrt(d_v d_u).  Consecutive threads write consecutive words.
// LEVELS: S holds the quantisation levels already (no scaled output), so the
// kept words are copied as they are.
// With only the kept output and r >= BS, thread t owns zig-zag positions
// t, t + BS, ... of every tile: it looks a position up once and walks the
// tiles, each step a coalesced run of BS words across the threads (measured
// +7 % on quantised int16 frames).  Otherwise consecutive threads take
// consecutive (tile, position) elements (with the scaled output as a second
// stream, the position-major order measured 5-13 % slower).
template <int KIND, int N, bool QUANT, bool LEVELS, int BS, int KB = N>
__device__ __forceinline__ void gather_outputs(const int* S, const Shared<N>& sh,
                                               const GroupIO& io) {
  using C = Cfg<N, BS, KB>;
  const int r = io.r;
  // largest r the kept bound allows; below BS the branch is not compiled
  constexpr int kMaxR = KB == N ? N * N : KB * (KB + 1) / 2;
  if (kMaxR >= BS && r >= BS && io.scaled == nullptr) {
    if (io.kept == nullptr) return;
    uint32_t* kept = reinterpret_cast<uint32_t*>(io.kept);
    for (int p = threadIdx.x; p < r; p += BS) {
      const int w = zz_word<KIND, N>(sh, p);
      const int off = w & 0xffff;
      const int32_t mq = QUANT && !LEVELS ? sh.mq[w >> 16] : 0;
      int e = p;
      for (int k = 0; k < io.nact; ++k, e += r) {
        const int val = S[__mul24(k, C::TS) + off];
        st_stream(kept + e, static_cast<uint32_t>(QUANT && !LEVELS ? quantise(val, mq) : val));
      }
    }
    return;
  }
  const int total = io.nact * r;
  if (threadIdx.x >= total) return;
  // quotients by r through one approximate reciprocal: for t <= 256 and
  // r <= 1024, (t + 1/2) / r lies at least 1/(2r) >= 2^-11 from an integer,
  // far more than the few ulps of error of the reciprocal and the product,
  // so the truncation is floor(t / r)
  const float rr = __builtin_amdgcn_rcpf(static_cast<float>(r));
  int k = static_cast<int>((static_cast<float>(threadIdx.x) + 0.5f) * rr);
  int p = threadIdx.x - k * r;
  const int dk = static_cast<int>((static_cast<float>(BS) + 0.5f) * rr), dp = BS - dk * r;
  for (int e = threadIdx.x; e < total; e += BS) {
    const int w = zz_word<KIND, N>(sh, p);
    const int val = S[__mul24(k, C::TS) + (w & 0xffff)];
    const int ci = w >> 16;
    if (io.kept != nullptr) {
      const int b = QUANT && !LEVELS ? quantise(val, sh.mq[ci]) : val;
      st_stream(reinterpret_cast<uint32_t*>(io.kept) + e, static_cast<uint32_t>(b));
    }
    if (io.scaled != nullptr)
      st_stream(reinterpret_cast<uint32_t*>(io.scaled) + e,
                __builtin_bit_cast(uint32_t, static_cast<float>(val) * sh.s2[ci]));
    p += dp;
    k += dk;
    if (p >= r) {
      p -= r;
      ++k;
    }
  }
}

// Row forward: load row i of tile k, transform it, store it transposed so that
// column j of tile k is contiguous: S[k][j][i].  Returns the row as loaded.
// Only columns j < KB are stored (the kept bound: no column >= KB keeps a
// coefficient), so the butterfly's other outputs are dead code.
template <int KIND, int N, int DT, int BS, int KB = N>
__device__ __forceinline__ void row_forward(int* S, const GroupIO& io, int i, int k,
                                            RowWords<N, DT>& x) {
  using C = Cfg<N, BS, KB>;
  load_row<N, DT>(io.src, io.tile_pix + static_cast<int64_t>(i) * io.pitch, io.active, x);
  int a[N];
  unpack_row<N, DT>(x, a);
  fwdN<KIND, N>(a);
#pragma unroll
  for (int j = 0; j < KB; ++j) S[k * C::TS + j * C::CS + i] = a[j];
}

// ------------------------------------------------------------ fused group
// Forward -> retain / quantise -> (outputs) -> inverse -> round -> store for
// the TPW tiles of one workgroup; returns this thread's squared
// reconstruction error (its row of its tile; 0 unless io.sse is set and the
// tile exists).  Every thread of the workgroup calls it; the tables in sh
// must have been written before it is called.  NT selects non-temporal
// reconstruction stores.  KB is a compile-time kept bound: every retained
// coefficient has v, u < KB (true when r <= KB (KB + 1) / 2, the zig-zag
// prefix of KB anti-diagonals), so the forward butterflies need only their
// first KB outputs and the inverse ones see zeros in their inputs >= KB; the
// compiler removes the additions that only feed or read those.
template <int KIND, int N, int DT, bool QUANT, int BS = kBlock, bool NT = true, int KB = N>
__device__ __forceinline__ unsigned long long compress_group(int* S, const Shared<N>& sh, const GroupIO& io) {
  using C = Cfg<N, BS, KB>;
  static_assert(!(QUANT && (N == 8 || KB != N)), "quantised groups: N = 16, 32 with the full bound");
  constexpr RowClasses<N> RC = row_classes<KIND, N>();
  const int a_idx = threadIdx.x / C::TPW;
  const int k = threadIdx.x % C::TPW;

  // phase 1: rows
  RowWords<N, DT> x;
  row_forward<KIND, N, DT, BS, KB>(S, io, a_idx, k, x);
  __syncthreads();

  // phase 2: columns, forward.  A column that keeps no coefficient (the
  // zig-zag prefix keeps rows 0 .. keep-1 of column j) is neither output nor
  // inverted: its transform is skipped, which whole waves do at small r
  // (a wave holds 64 / TPW consecutive columns).
  const int j = a_idx;
  int keep;
  if constexpr (keep_from_table<N, KB>())
    keep = j < KB ? kKeepRows8.c[min(io.r, 64)][j] : 0;
  else
    keep = j < KB ? sh.cnt[j] : 0;
  int c[N];
  if (keep > 0) {
    read_column<N, BS, KB>(S, j, k, c);
    fwdN<KIND, N>(c);
    if constexpr (DT == DT_U8)
      if (j == 0) c[0] -= 128 * N * N;   // level shift folded into the DC coefficient
  } else {
#pragma unroll
    for (int v = 0; v < N; ++v) c[v] = 0;
  }
  const int cls_u = sh.cls[j];
  double m_u[RC.count];
  int dq_u[RC.count];
  if constexpr (QUANT) {
#pragma unroll
    for (int q = 0; q < RC.count; ++q) {
      m_u[q] = quant_mult(sh.mq[q * 4 + cls_u]);
      dq_u[q] = sh.dq[q * 4 + cls_u];
    }
  }
  __syncthreads();  // S is free again

  // Outputs, then the zonal mask (a prefix of the column; nothing to mask
  // when every coefficient is kept) and the quantisation levels, in place: a
  // column holds one array of N values.  With the scaled values wanted the
  // coefficients are staged before that (the gather quantises the kept
  // ones itself); otherwise the levels (or the kept coefficients) after it.
  const bool outs = io.kept != nullptr || io.scaled != nullptr;
  if (outs && io.scaled != nullptr) {
    write_column_rows<N, BS, KB, KB>(S, j, k, c);   // [k][v][u], rows v < KB
    __syncthreads();
    gather_outputs<KIND, N, QUANT, false, BS, KB>(S, sh, io);
    __syncthreads();
  }
  if (KB == N && io.r >= N * N) {   // uniform: every coefficient kept
    if constexpr (QUANT) {
#pragma unroll
      for (int v = 0; v < N; ++v) c[v] = quantise_level(c[v], m_u[RC.cls[v]]);
    }
  } else {
#pragma unroll
    for (int v = 0; v < N; ++v) {
      const int b = v < KB && v < keep ? c[v] : 0;
      if constexpr (QUANT) c[v] = quantise_level(b, m_u[RC.cls[v]]);
      else c[v] = b;
    }
  }
  if (outs && io.scaled == nullptr) {
    write_column_rows<N, BS, KB, KB>(S, j, k, c);
    __syncthreads();
    gather_outputs<KIND, N, QUANT, QUANT, BS, KB>(S, sh, io);
    __syncthreads();
  }
  if (io.dst == nullptr && !io.sse) return 0ull;

  // dequantise
  if constexpr (QUANT) {
#pragma unroll
    for (int v = 0; v < N; ++v) c[v] = __mul24(c[v], dq_u[RC.cls[v]]);
  }

  // phase 2b: columns, inverse (a column with nothing kept stays zero)
  if (keep > 0) {
    invN<KIND, N>(c);
    if constexpr (QUANT) {
      // K = 2U: halve exactly so the second pass stays within 32 bits
#pragma unroll
      for (int v = 0; v < N; ++v) c[v] >>= 1;
    }
  }
  if (j < KB) write_inverse_column<N, BS, KB>(S, j, k, c);
  __syncthreads();

  // phase 3: rows, inverse (columns >= KB are zero)
  const int i = a_idx;
  int z[N];
  read_row<N, BS, KB>(S, i, k, z);
  invN<KIND, N>(z);
  // zonal: Z = 4 X, y = round(Z / (4 N^2)); quantised: Z = 2 X~, y = round(X~ / (2 N^2))
  const unsigned long long e = store_row<N, DT, C::SROUND, NT>(
      io.dst, io.tile_pix + static_cast<int64_t>(i) * io.pitch, io.active, z,
      io.sse ? &x : nullptr);
  __syncthreads();  // S may be reused by the caller
  return io.active ? e : 0ull;
}

}  // namespace jam
}  // namespace adct
