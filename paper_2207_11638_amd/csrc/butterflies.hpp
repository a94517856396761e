// Add-only fast algorithms of the Chen-based DCT approximations.
//
// Everything here is __host__ __device__ so that the library can build the
// transform matrices it computes (for self-checks) with exactly the code the
// kernels run.
//
// 8-point forward (sections 3, eqs. 4 and 5): x -> B8 -> M4 -> M3 -> M2 -> M1 -> P8.
//   Kind 1 (T~8, sign of Chen's constants) costs 26 additions, kind 2 (T^8,
//   round of the constants: alpha=1, beta=(1,1,1,0), gamma=(1,0)) costs 22.
// 8-point inverse (eqs. 6 and 7): T^-1 = 1/2 B8^T M4^-1 M3^-1 M2^-1 M1^T P8^T.
//   Each factor inverse is 1/2 times an integer matrix, so the code applies
//   the integer chain K8 = B8 (2 M4^-1) (2 M3^-1) (2 M2^-1) M1^T P8^T = 16 T8^-1.
// N-point (section 6.1): T_N = M_per diag(T_{N/2}, T_{N/2}) M_add, with
//   M_add = [[I, Ibar], [Ibar, -I]] (N additions) and M_per the interleave
//   (output 2k <- top half k, output 2k+1 <- bottom half k).  The inverse is
//   T_N^-1 = 1/2 M_add^T diag(T_{N/2}^-1, T_{N/2}^-1) M_per^T; the integer chain
//   K_N = M_add^T diag(K_{N/2}, K_{N/2}) M_per^T equals 2N T_N^-1.
// So for every N the integer inverse chain K_N is twice U_N = N T_N^-1.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__) || defined(__HIP__)
#include <hip/hip_runtime.h>
#define ADCT_HD __host__ __device__ __forceinline__ constexpr
#else
#define ADCT_HD inline constexpr
#endif

namespace adct {

// Transform ids: the two proposed approximations (section 3) and three of the
// 8-point comparison transforms of section 4 (Tables 1 and 2).
enum : int { KIND_SIGN = 1, KIND_ROUND = 2, KIND_WHT = 3, KIND_SDCT = 4, KIND_HT = 5 };

// ------------------------------------------- comparison transforms (N = 8)
// Walsh-Hadamard: three radix-2 stages (24 additions) give the Hadamard
// transform in Sylvester's natural row order (HT); the WHT lists the same
// rows by sequency (number of sign changes).  H H^T = 8 I, so the integer
// inverse chain 16 H^-1 is 2 H^T.
template <bool SEQUENCY>
ADCT_HD void hadamard8(int (&x)[8]) {
  int y[8] = {};
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    y[i] = x[i] + x[i + 4];
    y[i + 4] = x[i] - x[i + 4];
  }
  int z[8] = {};
#pragma unroll
  for (int h = 0; h < 2; ++h)
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      z[4 * h + i] = y[4 * h + i] + y[4 * h + i + 2];
      z[4 * h + i + 2] = y[4 * h + i] - y[4 * h + i + 2];
    }
  int n[8] = {};   // natural order: n[i] = sum_j (-1)^popcount(i & j) x[j]
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    n[2 * q] = z[2 * q] + z[2 * q + 1];
    n[2 * q + 1] = z[2 * q] - z[2 * q + 1];
  }
  if constexpr (SEQUENCY) {
    // natural row of sequency k: 0, 4, 6, 2, 3, 7, 5, 1
    x[0] = n[0]; x[1] = n[4]; x[2] = n[6]; x[3] = n[2];
    x[4] = n[3]; x[5] = n[7]; x[6] = n[5]; x[7] = n[1];
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) x[i] = n[i];
  }
}

template <bool SEQUENCY>
ADCT_HD void hadamard8_inv(int (&X)[8]) {
  int n[8] = {};
  if constexpr (SEQUENCY) {
    n[0] = X[0]; n[4] = X[1]; n[6] = X[2]; n[2] = X[3];
    n[3] = X[4]; n[7] = X[5]; n[5] = X[6]; n[1] = X[7];
  } else {
#pragma unroll
    for (int i = 0; i < 8; ++i) n[i] = X[i];
  }
  hadamard8<false>(n);   // H_natural is symmetric
#pragma unroll
  for (int i = 0; i < 8; ++i) X[i] = 2 * n[i];
}

// Signed DCT, sign(C8): the pre-additions B8 split x into sums s and
// differences d; the even rows are a 4-point Hadamard of s, the odd rows a
// 4-point chain on d (24 additions in all, Table 2).
ADCT_HD void sdct8(int (&x)[8]) {
  const int s0 = x[0] + x[7], s1 = x[1] + x[6], s2 = x[2] + x[5], s3 = x[3] + x[4];
  const int d0 = x[0] - x[7], d1 = x[1] - x[6], d2 = x[2] - x[5], d3 = x[3] - x[4];
  const int e0 = s0 + s3, e1 = s1 + s2, e2 = s0 - s3, e3 = s1 - s2;
  const int a = d0 - d1, b = d2 + d3, c = d2 - d3, p = d0 + d1;
  x[0] = e0 + e1;
  x[2] = e2 + e3;
  x[4] = e0 - e1;
  x[6] = e2 - e3;
  x[1] = p + b;
  x[3] = a - b;
  x[5] = a + b;
  x[7] = a + c;
}

// 16 sign(C8)^-1 = B8^T diag(2 E^T, 8 O^-1) with E the even 4-point Hadamard
// (E E^T = 4 I) and 8 O^-1 = 4 [[1,1,0,0],[1,0,-1,0],[0,-1,0,1],[0,0,1,-1]]
// for the odd rows.
ADCT_HD void sdct8_inv(int (&X)[8]) {
  const int f0 = X[0] + X[4], f1 = X[0] - X[4], f2 = X[2] + X[6], f3 = X[2] - X[6];
  const int s0 = 2 * (f0 + f2), s1 = 2 * (f1 + f3), s2 = 2 * (f1 - f3), s3 = 2 * (f0 - f2);
  const int d0 = 4 * (X[1] + X[3]), d1 = 4 * (X[1] - X[5]);
  const int d2 = 4 * (X[7] - X[3]), d3 = 4 * (X[5] - X[7]);
  X[0] = s0 + d0;
  X[1] = s1 + d1;
  X[2] = s2 + d2;
  X[3] = s3 + d3;
  X[4] = s3 - d3;
  X[5] = s2 - d2;
  X[6] = s1 - d1;
  X[7] = s0 - d0;
}

// ------------------------------------------------------------ 8-point forward
template <int KIND>
ADCT_HD void fwd8(int (&x)[8]) {
  if constexpr (KIND == KIND_WHT || KIND == KIND_HT) {
    hadamard8<KIND == KIND_WHT>(x);
    return;
  } else if constexpr (KIND == KIND_SDCT) {
    sdct8(x);
    return;
  }
  // B8: pre-additions
  const int y0 = x[0] + x[7], y1 = x[1] + x[6], y2 = x[2] + x[5], y3 = x[3] + x[4];
  const int y4 = x[3] - x[4], y5 = x[2] - x[5], y6 = x[1] - x[6], y7 = x[0] - x[7];
  // M4 = diag(B4, A3(alpha = 1))
  const int z0 = y0 + y3, z1 = y1 + y2, z2 = y1 - y2, z3 = y0 - y3;
  const int z4 = y7, z5 = y5 + y6, z6 = y6 - y5, z7 = y4;
  // M3 = diag(C~(alpha, gamma), A2)
  const int w0 = z0 + z1, w1 = z0 - z1;
  int w2 = 0, w3 = 0;
  if constexpr (KIND == KIND_SIGN) {  // gamma = (1, 1)
    w2 = z3 - z2;
    w3 = z2 + z3;
  } else {                            // gamma = (1, 0)
    w2 = -z2;
    w3 = z3;
  }
  const int w4 = z4 + z5, w5 = z4 - z5, w6 = z7 - z6, w7 = z6 + z7;
  // M2 = diag(P4, A1(beta))
  const int v0 = w0, v1 = w3, v2 = w1, v3 = w2;
  int v4 = 0, v7 = 0;
  if constexpr (KIND == KIND_SIGN) {  // beta = (1, 1, 1, 1)
    v4 = w4 + w7;
    v7 = w4 - w7;
  } else {                            // beta = (1, 1, 1, 0)
    v4 = w4;
    v7 = -w7;
  }
  const int v5 = w5 + w6, v6 = w5 - w6;
  // M1 = diag(I4, Ibar4 Q) followed by the output permutation P8
  x[0] = v0;
  x[1] = v4;
  x[2] = v1;
  x[3] = v6;
  x[4] = v2;
  x[5] = v5;
  x[6] = v3;
  x[7] = v7;
}

// ------------------------------------------------ 8-point inverse (K8 = 16 T^-1)
template <int KIND>
ADCT_HD void inv8(int (&X)[8]) {
  if constexpr (KIND == KIND_WHT || KIND == KIND_HT) {
    hadamard8_inv<KIND == KIND_WHT>(X);
    return;
  } else if constexpr (KIND == KIND_SDCT) {
    sdct8_inv(X);
    return;
  }
  // P8^T then M1^T
  const int v0 = X[0], v1 = X[2], v2 = X[4], v3 = X[6];
  const int v4 = X[1], v5 = X[5], v6 = X[3], v7 = X[7];
  // 2 M2^-1 = diag(2 P4^T, 2 A1^-1)
  const int w0 = 2 * v0, w1 = 2 * v2, w2 = 2 * v3, w3 = 2 * v1;
  int w4 = 0, w7 = 0;
  if constexpr (KIND == KIND_SIGN) {  // 2 A1^-1 = A1
    w4 = v4 + v7;
    w7 = v4 - v7;
  } else {                            // 2 A1^-1 = diag(2, [[1,1],[1,-1]], -2)
    w4 = 2 * v4;
    w7 = -2 * v7;
  }
  const int w5 = v5 + v6, w6 = v5 - v6;
  // 2 M3^-1
  const int z0 = w0 + w1, z1 = w0 - w1;
  int z2 = 0, z3 = 0;
  if constexpr (KIND == KIND_SIGN) {
    z2 = w3 - w2;
    z3 = w2 + w3;
  } else {
    z2 = -2 * w2;
    z3 = 2 * w3;
  }
  const int z4 = w4 + w5, z5 = w4 - w5, z6 = w7 - w6, z7 = w6 + w7;
  // 2 M4^-1 = diag(B4, [[0,0,0,2],[0,1,-1,0],[0,1,1,0],[2,0,0,0]])
  const int y0 = z0 + z3, y1 = z1 + z2, y2 = z1 - z2, y3 = z0 - z3;
  const int y4 = 2 * z7, y5 = z5 - z6, y6 = z5 + z6, y7 = 2 * z4;
  // B8 (B8^-1 = B8^T / 2 and B8^T = B8)
  X[0] = y0 + y7;
  X[1] = y1 + y6;
  X[2] = y2 + y5;
  X[3] = y3 + y4;
  X[4] = y3 - y4;
  X[5] = y2 - y5;
  X[6] = y1 - y6;
  X[7] = y0 - y7;
}

// ------------------------------------------------------ N-point (JAM) forward
template <int KIND, int N>
ADCT_HD void fwdN(int (&x)[N]) {
  if constexpr (N == 8) {
    fwd8<KIND>(x);
  } else {
    constexpr int H = N / 2;
    int u[H] = {}, w[H] = {};
#pragma unroll
    for (int i = 0; i < H; ++i) {
      u[i] = x[i] + x[N - 1 - i];       // top half of M_add
      w[i] = x[H - 1 - i] - x[H + i];   // bottom half of M_add
    }
    fwdN<KIND, H>(u);
    fwdN<KIND, H>(w);
#pragma unroll
    for (int k = 0; k < H; ++k) {       // M_per interleave
      x[2 * k] = u[k];
      x[2 * k + 1] = w[k];
    }
  }
}

// ------------------------------------------- N-point (JAM) inverse, K_N = 2N T^-1
template <int KIND, int N>
ADCT_HD void invN(int (&X)[N]) {
  if constexpr (N == 8) {
    inv8<KIND>(X);
  } else {
    constexpr int H = N / 2;
    int p[H] = {}, q[H] = {};
#pragma unroll
    for (int k = 0; k < H; ++k) {       // M_per^T
      p[k] = X[2 * k];
      q[k] = X[2 * k + 1];
    }
    invN<KIND, H>(p);
    invN<KIND, H>(q);
#pragma unroll
    for (int i = 0; i < H; ++i) {       // M_add^T = M_add
      X[i] = p[i] + q[H - 1 - i];
      X[H + i] = p[H - 1 - i] - q[i];
    }
  }
}

// ------------------------------------------------------------------ zig-zag
// Position of coefficient (v, u) (v vertical, u horizontal frequency) in the
// JPEG zig-zag scan of an N x N block: anti-diagonals d = v + u in increasing
// order, odd d scanned with increasing v, even d with decreasing v.
ADCT_HD int zz_pos(int n, int v, int u) {
  const int d = v + u;
  if (d < n) {
    const int base = d * (d + 1) / 2;
    return base + ((d & 1) ? v : u);
  }
  const int tail = (2 * n - 1 - d) * (2 * n - d) / 2;
  const int base = n * n - tail;
  return base + ((d & 1) ? v - (d - n + 1) : (n - 1 - v));
}

// Row classes of T_N: the distinct values of diag(T_N T_N^T), sorted
// increasingly, numbered 0, 1, ...; cls[v] is the class of row v.  Computed
// from the forward butterfly itself (at compile time in the kernels), so the
// host tables and the kernels agree by construction.
template <int N>
struct RowClasses {
  int cls[N];
  long long value[4];
  int count;
};

template <int KIND, int N>
ADCT_HD RowClasses<N> row_classes() {
  long long d[N] = {};
  for (int j = 0; j < N; ++j) {
    int e[N] = {};
    e[j] = 1;
    fwdN<KIND, N>(e);
    for (int v = 0; v < N; ++v) d[v] += static_cast<long long>(e[v]) * e[v];
  }
  RowClasses<N> rc{};
  rc.count = 0;
  for (int v = 0; v < N; ++v) {       // insertion of distinct values, kept sorted
    bool seen = false;
    for (int c = 0; c < rc.count; ++c) seen = seen || rc.value[c] == d[v];
    if (seen) continue;
    int c = rc.count++;
    while (c > 0 && rc.value[c - 1] > d[v]) {
      rc.value[c] = rc.value[c - 1];
      --c;
    }
    rc.value[c] = d[v];
  }
  for (int v = 0; v < N; ++v)
    for (int c = 0; c < rc.count; ++c)
      if (rc.value[c] == d[v]) rc.cls[v] = c;
  return rc;
}

// Rounded division by 2^S with the paper's round() (half away from zero):
// round(z / 2^S) = (z + 2^(S-1) - [z < 0]) >> S  (arithmetic shift = floor).
template <int S>
ADCT_HD int round_shift(int z) {
  return (z + (1 << (S - 1)) + (z >> 31)) >> S;
}

// Same, with a constant added to the quotient: round(z / 2^S) + OFF.
template <int S, int OFF>
ADCT_HD int round_shift_offset(int z) {
  return (z + (1 << (S - 1)) + (OFF << S) + (z >> 31)) >> S;
}

// round(z / 2^S) + 128 clipped to [0, 255].  The clip is applied to the
// dividend (floor(t / 2^S) clipped to [0, 255] equals floor(clip(t, 0,
// 2^(S+8) - 1) / 2^S)), followed by a logical shift: this form keeps the
// compiler from fusing shift, saturation and byte packing into one gfx950
// instruction whose upper result bits it wrongly assumes to be zero.
template <int S>
ADCT_HD int round_shift_u8(int z) {
  const int t = z + (1 << (S - 1)) + (128 << S) + (z >> 31);
  const int c = t < 0 ? 0 : (t > (256 << S) - 1 ? (256 << S) - 1 : t);
  return static_cast<int>(static_cast<unsigned>(c) >> S);
}

#if defined(__HIPCC__) || defined(__HIP__)
// Four results of round_shift_u8<S> packed into one word, byte b from z_b.
// Each clipped dividend holds its result in bits S .. S + 7 (byte 1 for
// S = 8, byte 0 after the shift otherwise); two byte permutes and an or
// gather the four bytes.
template <int S>
__device__ __forceinline__ uint32_t pack_round_u8(int z0, int z1, int z2, int z3) {
  const auto clip = [](int z) -> uint32_t {
    const int t = z + (1 << (S - 1)) + (128 << S) + (z >> 31);
    const int c = t < 0 ? 0 : (t > (256 << S) - 1 ? (256 << S) - 1 : t);
    return S == 8 ? static_cast<uint32_t>(c) : static_cast<uint32_t>(c) >> S;
  };
  constexpr uint32_t B = S == 8 ? 1u : 0u;   // byte holding the result
  const uint32_t lo = __builtin_amdgcn_perm(clip(z1), clip(z0), 0x0c0c0000u | ((4u + B) << 8) | B);
  const uint32_t hi = __builtin_amdgcn_perm(clip(z3), clip(z2), ((4u + B) << 24) | (B << 16) | 0x0c0cu);
  return lo | hi;
}

// Pointers into device memory, typed as the global address space.  Pixel
// and output pointers reach some kernels through tables in device memory
// (the serving kernels' request records), where the compiler cannot tell
// their address space and would emit flat accesses, which also count
// against the LDS wait counter; the shared load and store helpers go through
// these typed pointers, so every kernel gets global loads and stores.
template <class T>
using gptr = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ gptr<T> to_global(T* p) {
  return (gptr<T>)p;
}

// Loads and stores of the HIP vector types through global pointers (as
// native vectors: the class types have no assignment from the global
// address space).
typedef uint32_t u32x2_t __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint2 ld_global(const uint2* p) {
  const u32x2_t v = *to_global(reinterpret_cast<const u32x2_t*>(p));
  return make_uint2(v.x, v.y);
}
__device__ __forceinline__ uint4 ld_global(const uint4* p) {
  const u32x4_t v = *to_global(reinterpret_cast<const u32x4_t*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ void st_global(uint32_t* p, uint32_t v) { *to_global(p) = v; }
__device__ __forceinline__ void st_global(uint2* p, uint2 v) {
  *to_global(reinterpret_cast<u32x2_t*>(p)) = u32x2_t{v.x, v.y};
}
__device__ __forceinline__ void st_global(uint4* p, uint4 v) {
  *to_global(reinterpret_cast<u32x4_t*>(p)) = u32x4_t{v.x, v.y, v.z, v.w};
}

// Streaming stores: every output word is written once and not read again by
// the kernel, so the stores carry the non-temporal hint.
__device__ __forceinline__ void st_stream(uint32_t* p, uint32_t v) {
  __builtin_nontemporal_store(v, to_global(p));
}
__device__ __forceinline__ void st_stream(uint2* p, uint2 v) {
  const gptr<uint32_t> g = to_global(reinterpret_cast<uint32_t*>(p));
  __builtin_nontemporal_store(v.x, g);
  __builtin_nontemporal_store(v.y, g + 1);
}
__device__ __forceinline__ void st_stream(uint4* p, uint4 v) {
  const gptr<uint32_t> g = to_global(reinterpret_cast<uint32_t*>(p));
  __builtin_nontemporal_store(v.x, g);
  __builtin_nontemporal_store(v.y, g + 1);
  __builtin_nontemporal_store(v.z, g + 2);
  __builtin_nontemporal_store(v.w, g + 3);
}

// Non-temporal store when NT (whole lines written by one wave: the data is
// not read again), ordinary store otherwise (a row segment that shares its
// lines with tiles that another launch writes: the cache merges them).
template <bool NT, typename T>
__device__ __forceinline__ void st_pix(T* p, T v) {
  if constexpr (NT) st_stream(p, v);
  else st_global(p, v);
}
#endif

}  // namespace adct
