// Population storage formats.  Every format stores the shifted population
// h_i = f_i - w_i, so that the O(1) lattice weight does not consume mantissa
// bits (h_i is O(Ma) + O(rho - 1)); the kernels compute with h_i throughout.
// The 16-bit formats round to nearest even on store and widen to FP32 on load.
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace lbm {

enum StorageKind { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2, ST_BF16S = 3 };

template <int S>
struct Storage;

template <>
struct Storage<ST_F64> {
  using T = double;
  using R = double;
  template <class L>
  __device__ __forceinline__ static R load(const T* p, int) { return *p; }
  template <class L>
  __device__ __forceinline__ static void store(T* p, R v, int) { *p = v; }
};

template <>
struct Storage<ST_F32> {
  using T = float;
  using R = float;
  template <class L>
  __device__ __forceinline__ static R load(const T* p, int) { return *p; }
  template <class L>
  __device__ __forceinline__ static void store(T* p, R v, int) { *p = v; }
};

template <>
struct Storage<ST_F16S> {
  using T = __half;
  using R = float;
  template <class L>
  __device__ __forceinline__ static R load(const T* p, int) { return __half2float(*p); }
  template <class L>
  __device__ __forceinline__ static void store(T* p, R v, int) { *p = __float2half_rn(v); }
};

template <>
struct Storage<ST_BF16S> {
  using T = __hip_bfloat16;
  using R = float;
  template <class L>
  __device__ __forceinline__ static R load(const T* p, int) { return __bfloat162float(*p); }
  template <class L>
  __device__ __forceinline__ static void store(T* p, R v, int) { *p = __float2bfloat16(v); }
};

inline size_t storage_bytes(int s) { return s == ST_F64 ? 8 : s == ST_F32 ? 4 : 2; }
inline bool storage_is_f64(int s) { return s == ST_F64; }

}  // namespace lbm
