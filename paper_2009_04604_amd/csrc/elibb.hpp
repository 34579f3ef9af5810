// ELIBB interpolation weights in closed form (Sec. II.C-D).
//
// The missing population f_i(x_F, t+1) sits at link coordinate s = q; the
// interpolation points are placed at (eq. x_to_s_helper, resting-wall values)
//   P0  wall population at t+1              s = 0     weight a4
//   P1  post-collision wall population      s = 1     weight a5
//   P2  post-collision f_ibar(x_F)          s = 1 - q weight a2
//   P3  post-collision f_i(x_F)             s = 1 + q weight a3
// and the weights are the Lagrange basis over each variant's point set
// (eq. poli_coeff) evaluated at s = q, reduced to closed form:
//   U                 a4 = 1 - q,            a5 = q
//   F   (q < 1/2)     a4 = (1-2q)/(1-q),     a2 = q/(1-q)
//   F   (q >= 1/2)    a5 = (2q-1)/q,         a2 = (1-q)/q
//   UQ, FQ (q < 1/2)  a4 = 1-2q, a2 = 1,     a5 = 2q-1
//   FQ  (q >= 1/2)    a5 = (2q-1)/q^2, a2 = (1-q)/(2q^2), a3 = -(2q-1)(1-q)/(2q^2)
// UQ and FQ use F below the cutoff q_cut (0.01 in the paper).  HWBB: a2 = 1.
// (The F coefficients printed in the paper do not sum to one; these follow the
// Lagrange rule, which reproduces the printed BFL and ELIBB-U weights.)
#pragma once
#include "lattice.hpp"

namespace lbm {

enum Variant { FQ = 0, F = 1, UQ = 2, U = 3, HWBB = 4 };

template <typename T>
struct Coef {
  T a4, a5, a2, a3;
};

template <typename T>
LBM_HD Coef<T> elibb_coefficients(int variant, T q, T q_cut) {
  const T one = T(1), two = T(2), half = T(0.5);
  Coef<T> c{T(0), T(0), T(0), T(0)};
  if (variant == HWBB) {
    c.a2 = one;
    return c;
  }
  if (variant == U) {
    c.a4 = one - q;
    c.a5 = q;
    return c;
  }
  const bool linear = (variant == F) || (q < q_cut);
  if (linear) {
    if (q < half) {
      const T r = one / (one - q);
      c.a4 = (one - two * q) * r;
      c.a2 = q * r;
    } else {
      const T r = one / q;
      c.a5 = (two * q - one) * r;
      c.a2 = (one - q) * r;
    }
    return c;
  }
  if (variant == UQ || q < half) {
    c.a4 = one - two * q;
    c.a2 = one;
    c.a5 = two * q - one;
    return c;
  }
  // FQ, q >= 1/2
  const T r = one / (q * q);
  c.a5 = (two * q - one) * r;
  c.a2 = (one - q) * half * r;
  c.a3 = -(two * q - one) * (one - q) * half * r;
  return c;
}

#if defined(__HIPCC__)
// Branch-free form of elibb_coefficients for the kernels.  FP32 uses the
// hardware reciprocal (1 ulp); FP64 divides exactly.
template <typename T>
__device__ __forceinline__ T fast_recip(T x) {
  return T(1) / x;
}
#if defined(__HIP_DEVICE_COMPILE__)
template <>
__device__ __forceinline__ float fast_recip<float>(float x) {
  return __builtin_amdgcn_rcpf(x);
}
#endif

template <typename T>
__device__ __forceinline__ Coef<T> elibb_coefficients_fast(int variant, T q, T q_cut) {
  const T one = T(1), two = T(2), half = T(0.5);
  const T tq1 = two * q - one;                 // 2q - 1
  const T omq = one - q;                       // 1 - q
  const bool lo = q < half;
  // one reciprocal: 1 / (1 - q) below 1/2, 1 / q from 1/2 on (both >= 1/2)
  const T r = fast_recip(lo ? omq : q);
  // linear (ELIBB-F) weights
  const T fa4 = lo ? -tq1 * r : T(0);
  const T fa2 = lo ? q * r : omq * r;
  const T fa5 = lo ? T(0) : tq1 * r;
  // quadratic weights: UQ everywhere, FQ below 1/2 (r2 = 1 / q^2 where used)
  const T r2 = r * r;
  const bool fq_hi = (variant == FQ) && !lo;
  const T qa4 = fq_hi ? T(0) : -tq1;
  const T qa2 = fq_hi ? omq * half * r2 : one;
  const T qa5 = fq_hi ? tq1 * r2 : tq1;
  const T qa3 = fq_hi ? -tq1 * omq * half * r2 : T(0);
  Coef<T> c;
  if (variant == HWBB) {
    c = Coef<T>{T(0), T(0), one, T(0)};
  } else if (variant == U) {
    c = Coef<T>{omq, q, T(0), T(0)};
  } else {
    const bool linear = (variant == F) || (q < q_cut);
    c.a4 = linear ? fa4 : qa4;
    c.a5 = linear ? fa5 : qa5;
    c.a2 = linear ? fa2 : qa2;
    c.a3 = linear ? T(0) : qa3;
  }
  return c;
}
#endif  // __HIPCC__

// Wall-velocity term of a link.  With P0 = w rho e0 + n_pre,
// P1 = w rho e1 + n_post, P2 = f*_ibar + w rho m (eq. ELIBB-general, eq.
// ME-solid-to-fluid), e0 = f^eq_i(1, u_w(t+1)) / w_i, e1 = f^eq_i(1, u_w(t)) / w_i
// (eq. Eq2ndOrder), m = 2 c_i . u_w(t) / c_s^2, and the shifted populations
// h = f - w, the rebuilt population is
//   h_i(x_F, t+1) = a4 n_pre + a5 n_post + a2 h*_ibar + a3 h*_i
//                   + w_i [ (rho_F - 1)(a4 + a5) + rho_F Gw ],
//   Gw = a4 (e0 - 1) + a5 (e1 - 1) + a2 m        (zero for resting walls),
// using a2 + a3 + a4 + a5 = 1.
template <typename T>
LBM_HD T wall_term(const Coef<T>& c, T cu_t, T uu_t, T cu_t1, T uu_t1) {
  const T e0m1 = T(3) * cu_t1 + T(4.5) * cu_t1 * cu_t1 - T(1.5) * uu_t1;
  const T e1m1 = T(3) * cu_t + T(4.5) * cu_t * cu_t - T(1.5) * uu_t;
  const T m = T(6) * cu_t;
  return c.a4 * e0m1 + c.a5 * e1m1 + c.a2 * m;
}

}  // namespace lbm
