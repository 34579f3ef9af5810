// Population storage formats.  Every format stores the shifted population
// h_i = f_i - w_i, so that the O(1) lattice weight does not consume mantissa
// bits (h_i is O(Ma) + O(rho - 1)); the kernels compute with h_i throughout.
// The 16-bit formats widen to FP32 on load and round on store, to nearest even
// or stochastically (kinds ST_F16SR / ST_BF16SR: the node update's stores, with
// gfx950's stochastic-rounding conversions and a caller-supplied random word).
#pragma once
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include "lattice.hpp"

namespace lbm {

enum StorageKind { ST_F64 = 0, ST_F32 = 1, ST_F16S = 2, ST_BF16S = 3, ST_F16SR = 4, ST_BF16SR = 5 };

template <int S>
struct Storage;

template <>
struct Storage<ST_F64> {
  using T = double;
  using R = double;
  static constexpr bool stochastic = false;
  template <class L>
  __device__ __forceinline__ static R load(const T* p, int) { return *p; }
  template <class L>
  __device__ __forceinline__ static void store(T* p, R v, int) { *p = v; }
};

template <>
struct Storage<ST_F32> {
  using T = float;
  using R = float;
  static constexpr bool stochastic = false;
  template <class L>
  __device__ __forceinline__ static R load(const T* p, int) { return *p; }
  template <class L>
  __device__ __forceinline__ static void store(T* p, R v, int) { *p = v; }
};

template <>
struct Storage<ST_F16S> {
  using T = __half;
  using R = float;
  static constexpr bool stochastic = false;
  template <class L>
  __device__ __forceinline__ static R load(const T* p, int) { return __half2float(*p); }
  template <class L>
  __device__ __forceinline__ static void store(T* p, R v, int) { *p = __float2half_rn(v); }
};

template <>
struct Storage<ST_BF16S> {
  using T = __hip_bfloat16;
  using R = float;
  static constexpr bool stochastic = false;
  template <class L>
  __device__ __forceinline__ static R load(const T* p, int) { return __bfloat162float(*p); }
  template <class L>
  __device__ __forceinline__ static void store(T* p, R v, int) { *p = __float2bfloat16(v); }
};

// Stochastically rounded 16-bit stores: v_cvt_sr_{f16,bf16}_f32 rounds v up or
// down in magnitude with probabilities proportional to the distances, drawing
// on the random word `rnd`; loads are those of the nearest-even forms.
typedef _Float16 sr_f16x2 __attribute__((ext_vector_type(2)));
typedef __bf16 sr_bf16x2 __attribute__((ext_vector_type(2)));

template <>
struct Storage<ST_F16SR> : Storage<ST_F16S> {
  static constexpr bool stochastic = true;
  template <class L>
  __device__ __forceinline__ static void store(T* p, R v, int, uint32_t rnd) {
    // only the low half is stored, so the other half may hold anything: it is
    // v's own bits, which lets the conversion overwrite v's register in place
    const sr_f16x2 r = __builtin_amdgcn_cvt_sr_f16_f32(__builtin_bit_cast(sr_f16x2, v), v, rnd, false);
    *reinterpret_cast<uint16_t*>(p) = __builtin_bit_cast(uint16_t, r[0]);
  }
};

template <>
struct Storage<ST_BF16SR> : Storage<ST_BF16S> {
  static constexpr bool stochastic = true;
  template <class L>
  __device__ __forceinline__ static void store(T* p, R v, int, uint32_t rnd) {
    const sr_bf16x2 r = __builtin_amdgcn_cvt_sr_bf16_f32(__builtin_bit_cast(sr_bf16x2, v), v, rnd, false);
    *reinterpret_cast<uint16_t*>(p) = __builtin_bit_cast(uint16_t, r[0]);
  }
};

// The node update's store: stochastic where the kind says so, else the
// kind's own rounding (rnd unused).
template <int S, class L>
__device__ __forceinline__ void store_rounded(typename Storage<S>::T* p, typename Storage<S>::R v, int i, uint32_t rnd) {
  if constexpr (Storage<S>::stochastic) Storage<S>::template store<L>(p, v, i, rnd);
  else Storage<S>::template store<L>(p, v, i);
}

// Kind used by every kernel other than the step: the stored format of a
// stochastic kind is that of its nearest-even twin.
inline int storage_format(int s) { return s == ST_F16SR ? ST_F16S : (s == ST_BF16SR ? ST_BF16S : s); }

inline size_t storage_bytes(int s) { return s == ST_F64 ? 8 : s == ST_F32 ? 4 : 2; }
inline bool storage_is_f64(int s) { return s == ST_F64; }

}  // namespace lbm
