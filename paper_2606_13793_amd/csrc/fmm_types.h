// Compute types of the matrix-core kernels and how each stores, converts and
// multiplies its operands:
//   double     v_mfma_f64_16x16x4f64   K = 4 per op, FP64 accumulation
//   float      v_mfma_f32_16x16x4f32   K = 4 per op, FP32 accumulation
//   bf16_tag   v_mfma_f32_16x16x32_bf16 K = 32 per op (two interaction
//              offsets x 16 multipole terms), FP32 accumulation
// Included inside the kernels' namespace by fmm_impl.h.
#pragma once

typedef float f4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));  // 16 bytes of any element type
typedef __bf16 bf8 __attribute__((ext_vector_type(8)));

struct bf16_tag {};

template <typename CT>
struct Mf;
template <>
struct Mf<double> {
  using H = double;  // staged / tabulated element
  using AF = double;  // operand fragment of one lane
  using Acc = d4;
  static constexpr int KC = 4, OPM = 1, VPL = 1, IDX = 0;
  __device__ static Acc op(AF a, AF b, Acc c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
  // accumulator element v of a lane with k-group kq holds row:
  __device__ static int row(int v, int kq) { return 4 * v + kq; }
  template <typename E>
  __device__ __forceinline__ static AF frag(const E (&v)[1]) { return (double)v[0]; }
};
template <>
struct Mf<float> {
  using H = float;
  using AF = float;
  using Acc = f4;
  static constexpr int KC = 4, OPM = 1, VPL = 1, IDX = 1;
  __device__ static Acc op(AF a, AF b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
  __device__ static int row(int v, int kq) { return 4 * kq + v; }
  template <typename E>
  __device__ __forceinline__ static AF frag(const E (&v)[1]) { return (float)v[0]; }
};
template <>
struct Mf<bf16_tag> {
  using H = __bf16;
  using AF = bf8;
  using Acc = f4;
  static constexpr int KC = 16, OPM = 2, VPL = 8, IDX = 2;
  __device__ static Acc op(AF a, AF b, Acc c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
  __device__ static int row(int v, int kq) { return 4 * kq + v; }
  // (round to nearest even; a float converts to the same bf16 directly or
  // through double, which holds it exactly)
  template <typename E>
  __device__ __forceinline__ static AF frag(const E (&v)[8]) {
    AF f;
#pragma unroll
    for (int e = 0; e < 8; ++e) f[e] = static_cast<__bf16>(v[e]);
    return f;
  }
};

// Stores one chunk of N consecutive terms, converted to H with round to
// nearest even, at p (aligned to N elements) in one vector store: the typed
// multipole copies of mixed plans.
template <typename H, int N>
__device__ __forceinline__ void store_chunk(H* p, const double (&v)[N]) {
  typedef H vN __attribute__((ext_vector_type(N)));
  vN x;
#pragma unroll
  for (int e = 0; e < N; ++e) x[e] = static_cast<H>(v[e]);
  *reinterpret_cast<vN*>(p) = x;
}
