// Per-subelement integration of the LOR H(curl) matrix: the lowest-order
// Nedelec element on one trilinear subelement (Section 2.3: the lowest-order
// interpolation-histopolation space is the standard lowest-order Nedelec
// space on the refined mesh), 2x2x2 Gauss points q, weight 1/8.
//
// Reference edges (local +axis orientation): x-edges (b,c) -> b + 2c, y-edges
// (a,c) -> 4 + a + 2c, z-edges (a,b) -> 8 + a + 2b, with
//   n_x(b,c) = (l_b(eta) l_c(zeta), 0, 0),   curl = (0, s_c l_b(eta), -s_b l_c(zeta)),
//   n_y(a,c) = (0, l_a(xi) l_c(zeta), 0),    curl = (-s_c l_a(xi), 0, s_a l_c(zeta)),
//   n_z(a,b) = (0, 0, l_a(xi) l_b(eta)),     curl = (s_b l_a(xi), -s_a l_b(eta), 0),
// s_t = 2t - 1.  Covariant Piola: N = J^-T n, curl N = J curl n / det J, so
//   M_ab = beta  sum_q (1/8 det J) n_a^T (R R^T) n_b      (R rows: cofactor rows)
//   K_ab = kappa sum_q (1/8 det J) c_a^T (J^T J) c_b.
// The mass therefore reuses the H1 stiffness factor tables computed with beta
// (n_a has one nonzero component, exactly like one component of an H1
// gradient), and the curl-curl needs only one- and two-dimensional factors of
// Gamma = (kappa / 8 det J) J^T J:
//   D00[A] = sum G00 LL_A(xi), C11[B] = sum G11 LL_B(eta), C22[C] = sum G22 LL_C(zeta),
//   E01[x][y] = sum G01 l_x(xi) l_y(eta), D02[x][z] = sum G02 l_x(xi) l_z(zeta),
//   C12[y][z] = sum G12 l_y(eta) l_z(zeta).
#pragma once

#include "lor_h1_math.hpp"

namespace lor {

template <typename R>
struct NDCurl {
  R D00[3], C11[3], C22[3];
  R E01[2][2], D02[2][2], C12[2][2];
};

// Mass factor tables (H1Factors with beta, TM unused) and curl factors of one
// subelement; returns false if det J <= 0 at a Gauss point.
template <typename R>
__device__ __forceinline__ bool nd_factors(const R (&ex)[2][2][3], const R (&ey)[2][2][3], const R (&ez)[2][2][3],
                                           R kap, R bet, H1Factors<R>& F, NDCurl<R>& W) {
  R c0[2][2][3], c1[2][2][3], c2[2][2][3];
  jac_columns<R>(ex, ey, ez, c0, c1, c2);
  R H00[2][2] = {}, H11[2][2] = {}, H22[2][2] = {};
  R Z01[2][2][2] = {}, Z02[2][2][2] = {};
  R G12q[2][2][2];
  R P00[2] = {}, P11[2] = {}, P22[2] = {};
  R P01[2][2] = {}, P02[2][2] = {}, P12[2][2] = {};
  bool ok = true;
  const R wk = R(0.125) * kap;
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
        R r0[3], r1[3], r2[3];
        r0[0] = B[1] * C[2] - B[2] * C[1];
        r0[1] = B[2] * C[0] - B[0] * C[2];
        r0[2] = B[0] * C[1] - B[1] * C[0];
        r1[0] = C[1] * A[2] - C[2] * A[1];
        r1[1] = C[2] * A[0] - C[0] * A[2];
        r1[2] = C[0] * A[1] - C[1] * A[0];
        r2[0] = A[1] * B[2] - A[2] * B[1];
        r2[1] = A[2] * B[0] - A[0] * B[2];
        r2[2] = A[0] * B[1] - A[1] * B[0];
        const R det = A[0] * r0[0] + A[1] * r0[1] + A[2] * r0[2];
        ok = ok && (det > R(0));
        const R idet = rcp_refined(det);
        const R fb = wb * idet;
        const R fk = wk * idet;
        // mass metric (beta / 8 det) R R^T
        H00[q2][q3] += fb * (r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
        H11[q1][q3] += fb * (r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
        H22[q1][q2] += fb * (r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2]);
        const R h01 = fb * (r0[0] * r1[0] + r0[1] * r1[1] + r0[2] * r1[2]);
        const R h02 = fb * (r0[0] * r2[0] + r0[1] * r2[1] + r0[2] * r2[2]);
        G12q[q1][q2][q3] = fb * (r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2]);
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          Z01[x][q2][q3] += R(L1(x, q1)) * h01;
          Z02[x][q2][q3] += R(L1(x, q1)) * h02;
        }
        // curl metric (kappa / 8 det) J^T J
        P00[q1] += fk * (A[0] * A[0] + A[1] * A[1] + A[2] * A[2]);
        P11[q2] += fk * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
        P22[q3] += fk * (C[0] * C[0] + C[1] * C[1] + C[2] * C[2]);
        P01[q1][q2] += fk * (A[0] * B[0] + A[1] * B[1] + A[2] * B[2]);
        P02[q1][q3] += fk * (A[0] * C[0] + A[1] * C[1] + A[2] * C[2]);
        P12[q2][q3] += fk * (B[0] * C[0] + B[1] * C[1] + B[2] * C[2]);
      }
  h1_contract_stiffness<R>(H00, H11, H22, Z01, Z02, G12q, F);
#pragma unroll
  for (int A = 0; A < 3; ++A) {
    W.D00[A] = R(LL(A, 0)) * P00[0] + R(LL(A, 1)) * P00[1];
    W.C11[A] = R(LL(A, 0)) * P11[0] + R(LL(A, 1)) * P11[1];
    W.C22[A] = R(LL(A, 0)) * P22[0] + R(LL(A, 1)) * P22[1];
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      W.E01[x][y] = R(L1(x, 0)) * (R(L1(y, 0)) * P01[0][0] + R(L1(y, 1)) * P01[0][1]) +
                    R(L1(x, 1)) * (R(L1(y, 0)) * P01[1][0] + R(L1(y, 1)) * P01[1][1]);
      W.D02[x][y] = R(L1(x, 0)) * (R(L1(y, 0)) * P02[0][0] + R(L1(y, 1)) * P02[0][1]) +
                    R(L1(x, 1)) * (R(L1(y, 0)) * P02[1][0] + R(L1(y, 1)) * P02[1][1]);
      W.C12[x][y] = R(L1(x, 0)) * (R(L1(y, 0)) * P12[0][0] + R(L1(y, 1)) * P12[0][1]) +
                    R(L1(x, 1)) * (R(L1(y, 0)) * P12[1][0] + R(L1(y, 1)) * P12[1][1]);
    }
  return ok;
}

// Index of the unordered edge pair (u <= v) among the 78 pairs, u-major.
__host__ __device__ constexpr int pair_index12(int u, int v) {
  return u <= v ? 12 * u - (u * (u - 1)) / 2 + (v - u) : 12 * v - (v * (v - 1)) / 2 + (u - v);
}

// Entry (u, v), u <= v, of K + M in the local (+axis) orientation.
template <typename R>
__device__ __forceinline__ R nd_entry(const H1Factors<R>& F, const NDCurl<R>& W, int u, int v) {
  const int du = u >> 2, dv = v >> 2;   // 0: x-edge, 1: y-edge, 2: z-edge (du <= dv)
  const int p0 = u & 1, p1 = (u >> 1) & 1, q0 = v & 1, q1 = (v >> 1) & 1;
  auto sg = [](int t) { return t ? R(1) : R(-1); };
  if (du == 0 && dv == 0) {  // x(b,c)-x(b',c')
    const int b = p0, c = p1, b2 = q0, c2 = q1;
    return F.S0[b + b2][c + c2] + sg(c) * sg(c2) * W.C11[b + b2] + sg(b) * sg(b2) * W.C22[c + c2] -
           sg(c) * sg(b2) * W.C12[b][c2] - sg(b) * sg(c2) * W.C12[b2][c];
  }
  if (du == 1 && dv == 1) {  // y(a,c)-y(a',c')
    const int a = p0, c = p1, a2 = q0, c2 = q1;
    return F.S1[a + a2][c + c2] + sg(c) * sg(c2) * W.D00[a + a2] + sg(a) * sg(a2) * W.C22[c + c2] -
           sg(c) * sg(a2) * W.D02[a][c2] - sg(a) * sg(c2) * W.D02[a2][c];
  }
  if (du == 2 && dv == 2) {  // z(a,b)-z(a',b')
    const int a = p0, b = p1, a2 = q0, b2 = q1;
    return F.S2[a + a2][b + b2] + sg(b) * sg(b2) * W.D00[a + a2] + sg(a) * sg(a2) * W.C11[b + b2] -
           sg(b) * sg(a2) * W.E01[a][b2] - sg(a) * sg(b2) * W.E01[a2][b];
  }
  if (du == 0 && dv == 1) {  // x(b,c)-y(a',c')
    const int b = p0, c = p1, a2 = q0, c2 = q1;
    return F.T01[a2][b][c + c2] - sg(c) * sg(c2) * W.E01[a2][b] + sg(c) * sg(a2) * W.C12[b][c2] +
           sg(b) * sg(c2) * W.D02[a2][c] - sg(b) * sg(a2) * W.C22[c + c2];
  }
  if (du == 0 && dv == 2) {  // x(b,c)-z(a',b')
    const int b = p0, c = p1, a2 = q0, b2 = q1;
    return F.T02[a2][c][b + b2] + sg(c) * sg(b2) * W.E01[a2][b] - sg(c) * sg(a2) * W.C11[b + b2] -
           sg(b) * sg(b2) * W.D02[a2][c] + sg(b) * sg(a2) * W.C12[b2][c];
  }
  // y(a,c)-z(a',b')
  const int a = p0, c = p1, a2 = q0, b2 = q1;
  return F.T12[b2][c][a + a2] - sg(c) * sg(b2) * W.D00[a + a2] + sg(c) * sg(a2) * W.E01[a][b2] +
         sg(a) * sg(b2) * W.D02[a2][c] - sg(a) * sg(a2) * W.C12[b2][c];
}

}  // namespace lor
