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
