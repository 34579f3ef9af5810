// Velocity sets (D2Q9, D3Q19, D3Q27) as compile-time tables usable in host and device
// code.  c_s^2 = 1/3 (Sec. II.A).  Every loop over directions in the kernels is
// fully unrolled, so the switch statements below fold to constants.
#pragma once
#include <cstdint>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define LBM_HD __host__ __device__ __forceinline__
#else
#define LBM_HD inline
#endif

struct D2Q9 {
  static constexpr int Q = 9;
  static constexpr int D = 2;
  static constexpr int ID = 0;
  LBM_HD static constexpr int cx(int i) {
    return i == 1 || i == 5 || i == 6 ? 1 : (i == 2 || i == 7 || i == 8 ? -1 : 0);
  }
  LBM_HD static constexpr int cy(int i) {
    return i == 3 || i == 5 || i == 7 ? 1 : (i == 4 || i == 6 || i == 8 ? -1 : 0);
  }
  LBM_HD static constexpr int cz(int) { return 0; }
  LBM_HD static constexpr int opp(int i) {
    return i == 0 ? 0 : i == 1 ? 2 : i == 2 ? 1 : i == 3 ? 4 : i == 4 ? 3 : i == 5 ? 8 : i == 6 ? 7 : i == 7 ? 6 : 5;
  }
  LBM_HD static constexpr double w(int i) { return i == 0 ? 4.0 / 9.0 : (i <= 4 ? 1.0 / 9.0 : 1.0 / 36.0); }
};

struct D3Q19 {
  static constexpr int Q = 19;
  static constexpr int D = 3;
  static constexpr int ID = 1;
  // 1..6 axis; 7..10 (x,y); 11..14 (x,z); 15..18 (y,z); pair signs (+,+),(+,-),(-,+),(-,-)
  LBM_HD static constexpr int first_sign(int i) { return ((i - 7) % 4) < 2 ? 1 : -1; }
  LBM_HD static constexpr int second_sign(int i) { return ((i - 7) % 2) == 0 ? 1 : -1; }
  LBM_HD static constexpr int cx(int i) {
    return i == 1 ? 1 : i == 2 ? -1 : (i >= 7 && i <= 14) ? first_sign(i) : 0;
  }
  LBM_HD static constexpr int cy(int i) {
    return i == 3 ? 1 : i == 4 ? -1 : (i >= 7 && i <= 10) ? second_sign(i) : (i >= 15 ? first_sign(i) : 0);
  }
  LBM_HD static constexpr int cz(int i) {
    return i == 5 ? 1 : i == 6 ? -1 : (i >= 11 && i <= 14) ? second_sign(i) : (i >= 15 ? second_sign(i) : 0);
  }
  LBM_HD static constexpr int opp(int i) {
    return i == 0 ? 0 : (i <= 6 ? ((i % 2) ? i + 1 : i - 1) : (7 + 4 * ((i - 7) / 4) + (3 - (i - 7) % 4)));
  }
  LBM_HD static constexpr double w(int i) { return i == 0 ? 1.0 / 3.0 : (i <= 6 ? 1.0 / 18.0 : 1.0 / 36.0); }
};

struct D3Q27 {
  static constexpr int Q = 27;
  static constexpr int D = 3;
  static constexpr int ID = 2;
  // 0..18 as D3Q19; 19..26 the corners (+-1,+-1,+-1) in sign order
  // (+,+,+),(+,+,-),(+,-,+),(+,-,-),(-,+,+),(-,+,-),(-,-,+),(-,-,-)
  LBM_HD static constexpr int corner(int i, int bit) { return ((i - 19) >> bit) & 1 ? -1 : 1; }
  LBM_HD static constexpr int cx(int i) { return i >= 19 ? corner(i, 2) : D3Q19::cx(i); }
  LBM_HD static constexpr int cy(int i) { return i >= 19 ? corner(i, 1) : D3Q19::cy(i); }
  LBM_HD static constexpr int cz(int i) { return i >= 19 ? corner(i, 0) : D3Q19::cz(i); }
  LBM_HD static constexpr int opp(int i) { return i >= 19 ? 45 - i : D3Q19::opp(i); }
  LBM_HD static constexpr double w(int i) {
    return i == 0 ? 8.0 / 27.0 : (i <= 6 ? 2.0 / 27.0 : (i <= 18 ? 1.0 / 54.0 : 1.0 / 216.0));
  }
};

// Compile-time self-checks of the tables.
template <class L>
constexpr bool lattice_tables_ok() {
  double sw = 0.0;
  for (int i = 0; i < L::Q; ++i) {
    sw += L::w(i);
    if (L::cx(L::opp(i)) != -L::cx(i) || L::cy(L::opp(i)) != -L::cy(i) || L::cz(L::opp(i)) != -L::cz(i)) return false;
    if (L::opp(L::opp(i)) != i) return false;
  }
  return sw > 1.0 - 1e-15 && sw < 1.0 + 1e-15;
}
static_assert(lattice_tables_ok<D2Q9>(), "D2Q9 table");
static_assert(lattice_tables_ok<D3Q19>(), "D3Q19 table");
static_assert(lattice_tables_ok<D3Q27>(), "D3Q27 table");
