// Per-subelement integration of the LOR H(div) matrix: the lowest-order
// Raviart-Thomas element on one trilinear subelement (Section 2.3: the
// lowest-order interpolation-histopolation space is the standard lowest-order
// Raviart-Thomas space on the refined mesh), 2x2x2 Gauss points q, weight 1/8.
//
// Reference faces (local +axis normals): x-faces (xi = t) -> t, y-faces
// (eta = t) -> 2 + t, z-faces (zeta = t) -> 4 + t, with
//   n_x,t = (l_t(xi), 0, 0), n_y,t = (0, l_t(eta), 0), n_z,t = (0, 0, l_t(zeta)),
//   div n = s_t = 2t - 1.
// Contravariant Piola: N = J n / det J, div N = div n / det J, so
//   M_ab = beta  sum_q (1/8 det J) n_a^T (J^T J) n_b,
//   D_ab = kappa s_a s_b sum_q 1 / (8 det J).
// n_a has one nonzero component, a function of one coordinate, so the mass
// needs only one- and two-dimensional factors of Gamma = (beta / 8 det J) J^T J
// -- the same tables as the Nedelec curl-curl, with beta in place of kappa:
//   D00[A] = sum G00 LL_A(xi),  C11[B] = sum G11 LL_B(eta),  C22[C] = sum G22 LL_C(zeta),
//   E01[x][y] = sum G01 l_x(xi) l_y(eta), D02[x][z] = ..., C12[y][z] = ....
#pragma once

#include "lor_h1_math.hpp"

namespace lor {

template <typename R>
struct RTFactors {
  R D00[3], C11[3], C22[3];
  R E01[2][2], D02[2][2], C12[2][2];
  R W;  // sum_q 1 / (8 det J), times kappa
};

// Factor tables of one subelement; returns false if det J <= 0 at a Gauss point.
template <typename R>
__device__ __forceinline__ bool rt_factors(const R (&ex)[2][2][3], const R (&ey)[2][2][3], const R (&ez)[2][2][3],
                                           R kap, R bet, RTFactors<R>& F) {
  R c0[2][2][3], c1[2][2][3], c2[2][2][3];
  jac_columns<R>(ex, ey, ez, c0, c1, c2);
  R P00[2] = {}, P11[2] = {}, P22[2] = {};
  R P01[2][2] = {}, P02[2][2] = {}, P12[2][2] = {};
  R wsum = R(0);
  bool ok = true;
  const R wb = R(0.125) * bet;
#pragma unroll
  for (int q3 = 0; q3 < 2; ++q3)
#pragma unroll
    for (int q2 = 0; q2 < 2; ++q2)
#pragma unroll
      for (int q1 = 0; q1 < 2; ++q1) {
        const R* A = c0[q2][q3];
        const R* B = c1[q1][q3];
        const R* C = c2[q1][q2];
        const R det = A[0] * (B[1] * C[2] - B[2] * C[1]) + A[1] * (B[2] * C[0] - B[0] * C[2]) +
                      A[2] * (B[0] * C[1] - B[1] * C[0]);
        ok = ok && (det > R(0));
        const R idet = rcp_refined(det);
        wsum += idet;
        const R g = wb * idet;
        P00[q1] += g * (A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
        P11[q2] += g * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
        P22[q3] += g * (C[0] * C[0] + C[1] * C[1] + C[2] * C[2]);
        P01[q1][q2] += g * (A[0] * B[0] + A[1] * B[1] + A[2] * B[2]);
        P02[q1][q3] += g * (A[0] * C[0] + A[1] * C[1] + A[2] * C[2]);
        P12[q2][q3] += g * (B[0] * C[0] + B[1] * C[1] + B[2] * C[2]);
      }
  F.W = R(0.125) * kap * wsum;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    F.D00[a] = R(LL(a, 0)) * P00[0] + R(LL(a, 1)) * P00[1];
    F.C11[a] = R(LL(a, 0)) * P11[0] + R(LL(a, 1)) * P11[1];
    F.C22[a] = R(LL(a, 0)) * P22[0] + R(LL(a, 1)) * P22[1];
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      F.E01[x][y] = R(L1(x, 0)) * (R(L1(y, 0)) * P01[0][0] + R(L1(y, 1)) * P01[0][1]) +
                    R(L1(x, 1)) * (R(L1(y, 0)) * P01[1][0] + R(L1(y, 1)) * P01[1][1]);
      F.D02[x][y] = R(L1(x, 0)) * (R(L1(y, 0)) * P02[0][0] + R(L1(y, 1)) * P02[0][1]) +
                    R(L1(x, 1)) * (R(L1(y, 0)) * P02[1][0] + R(L1(y, 1)) * P02[1][1]);
      F.C12[x][y] = R(L1(x, 0)) * (R(L1(y, 0)) * P12[0][0] + R(L1(y, 1)) * P12[0][1]) +
                    R(L1(x, 1)) * (R(L1(y, 0)) * P12[1][0] + R(L1(y, 1)) * P12[1][1]);
    }
  return ok;
}

// Index of the unordered face pair (u <= v) among the 21 pairs, u-major.
__host__ __device__ constexpr int pair_index6(int u, int v) {
  return u <= v ? 6 * u - (u * (u - 1)) / 2 + (v - u) : 6 * v - (v * (v - 1)) / 2 + (u - v);
}

// Entry (u, v), u <= v, of kappa D + beta M in the local (+axis) orientation.
template <typename R>
__device__ __forceinline__ R rt_entry(const RTFactors<R>& F, int u, int v) {
  const int du = u >> 1, dv = v >> 1, t = u & 1, t2 = v & 1;
  const R div = (t == t2) ? F.W : -F.W;  // s_t s_t' W
  if (du == dv) {
    if (du == 0) return F.D00[t + t2] + div;
    if (du == 1) return F.C11[t + t2] + div;
    return F.C22[t + t2] + div;
  }
  if (du == 0 && dv == 1) return F.E01[t][t2] + div;
  if (du == 0 && dv == 2) return F.D02[t][t2] + div;
  return F.C12[t][t2] + div;
}

}  // namespace lor
