// Oracle (test infrastructure only): explicit SU(3) colour algebra with
// numeric Gell-Mann matrices, T^a = lambda^a / 2, Tr(T^a T^b) = delta^ab / 2,
// [T^a, T^b] = i f^abc T^c.  Everything is computed by brute force from the
// 3x3 matrices; nothing here is symbolic.  This is the "color algebra" part
// of the matrix element named in section 3 of the paper.
#pragma once
#include <array>
#include <cmath>
#include <complex>
#include <vector>

namespace oracle {

using cd = std::complex<double>;
using Mat3 = std::array<std::array<cd, 3>, 3>;

inline Mat3 mat3_zero() { return Mat3{}; }
inline Mat3 mat3_identity() {
  Mat3 m{};
  for (int i = 0; i < 3; ++i) m[i][i] = 1.0;
  return m;
}
inline Mat3 mat3_mul(const Mat3& a, const Mat3& b) {
  Mat3 m{};
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k) m[i][j] += a[i][k] * b[k][j];
  return m;
}

struct ColourTables {
  Mat3 T[8];
  double f[8][8][8];
  ColourTables() {
    const cd I(0, 1);
    for (int a = 0; a < 8; ++a) T[a] = Mat3{};
    // lambda^1 .. lambda^8 (Gell-Mann), then halved
    T[0][0][1] = 1.0; T[0][1][0] = 1.0;
    T[1][0][1] = -I;  T[1][1][0] = I;
    T[2][0][0] = 1.0; T[2][1][1] = -1.0;
    T[3][0][2] = 1.0; T[3][2][0] = 1.0;
    T[4][0][2] = -I;  T[4][2][0] = I;
    T[5][1][2] = 1.0; T[5][2][1] = 1.0;
    T[6][1][2] = -I;  T[6][2][1] = I;
    const double r3 = 1.0 / std::sqrt(3.0);
    T[7][0][0] = r3; T[7][1][1] = r3; T[7][2][2] = -2.0 * r3;
    for (int a = 0; a < 8; ++a)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) T[a][i][j] *= 0.5;
    // f^abc = -2 i Tr(T^a [T^b, T^c])
    for (int a = 0; a < 8; ++a)
      for (int b = 0; b < 8; ++b)
        for (int c = 0; c < 8; ++c) {
          const Mat3 bc = mat3_mul(T[b], T[c]);
          const Mat3 cb = mat3_mul(T[c], T[b]);
          cd tr = 0;
          for (int i = 0; i < 3; ++i)
            for (int k = 0; k < 3; ++k) tr += T[a][i][k] * (bc[k][i] - cb[k][i]);
          const cd val = cd(0, -2) * tr;
          f[a][b][c] = std::fabs(val.real()) < 1e-15 ? 0.0 : val.real();
        }
  }
};

inline const ColourTables& colour_tables() {
  static const ColourTables t;
  return t;
}

}  // namespace oracle
