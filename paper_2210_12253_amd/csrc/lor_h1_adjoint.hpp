// Adjoint of the per-subelement H1 integration (lor_h1_math.hpp).
//
// Given the adjoints of the 36 unique stiffness entries (computed with kappa = 1)
// and of the 36 unique mass entries (computed with beta), return the adjoints
// of the 12 edge vectors.  Each forward step is linear in the previous one
// except the per-point geometry, whose reverse is written out:
//   G_rc = f (r_r . r_c),  f = 1 / (8 det J),   D = beta det J / 8,
//   det J = J_0 . r_0,  r_0 = J_1 x J_2,  r_1 = J_2 x J_0,  r_2 = J_0 x J_1,
// so with d_rc = r_r . r_c:
//   fbar = sum_rc Gbar_rc d_rc,   dbar_rc = f Gbar_rc,
//   rbar_0 = 2 dbar_00 r_0 + dbar_01 r_1 + dbar_02 r_2   (and cyclically),
//   detbar = -fbar f / det + Dbar beta / 8,
//   and for r = a x b:  abar += b x rbar,  bbar += rbar x a.
// The factor contractions are transposed one axis at a time, like the forward.
#pragma once

#include "lor_h1_math.hpp"

namespace lor {

template <typename R>
__device__ __forceinline__ void cross_acc(const R* a, const R* b, R* out) {  // out += a x b
  out[0] += a[1] * b[2] - a[2] * b[1];
  out[1] += a[2] * b[0] - a[0] * b[2];
  out[2] += a[0] * b[1] - a[1] * b[0];
}

// Wk: adjoint of K (kappa = 1) per unique pair; Wm: adjoint of M per unique pair.
// Returns the adjoints of ex, ey, ez (overwritten).
template <typename R>
__device__ __forceinline__ void h1_adjoint(const R (&ex)[2][2][3], const R (&ey)[2][2][3], const R (&ez)[2][2][3],
                                           const R (&Wk)[36], const R (&Wm)[36], R bet, R (&gx)[2][2][3],
                                           R (&gy)[2][2][3], R (&gz)[2][2][3]) {
  // ---- mass: entries -> TM -> per-point D
  R Dbar[2][2][2];
  {
    R TMb[3][3][3] = {};
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = u; v < 8; ++v)
        TMb[(u & 1) + (v & 1)][((u >> 1) & 1) + ((v >> 1) & 1)][(u >> 2) + (v >> 2)] += Wm[pair_index(u, v)];
#pragma unroll
    for (int t1 = 0; t1 < 2; ++t1)
#pragma unroll
      for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
        for (int t3 = 0; t3 < 2; ++t3) {
          R acc = R(0);
#pragma unroll
          for (int A = 0; A < 3; ++A)
#pragma unroll
            for (int B = 0; B < 3; ++B)
#pragma unroll
              for (int C = 0; C < 3; ++C) acc += R(LL(A, t1) * LL(B, t2) * LL(C, t3)) * TMb[A][B][C];
          Dbar[t1][t2][t3] = acc;
        }
  }
  // ---- stiffness: entries -> factor adjoints -> per-point adjoints
  R H00b[2][2] = {}, H11b[2][2] = {}, H22b[2][2] = {};
  R Z01b[2][2][2] = {}, Z02b[2][2][2] = {}, G12b[2][2][2] = {};
  {
    H1Factors<R> Fb;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Fb.S0[i][j] = Fb.S1[i][j] = Fb.S2[i][j] = R(0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int k = 0; k < 3; ++k) Fb.T01[i][j][k] = Fb.T02[i][j][k] = Fb.T12[i][j][k] = R(0);
#pragma unroll
    for (int u = 0; u < 8; ++u)
#pragma unroll
      for (int v = u; v < 8; ++v) {
        const R w = Wk[pair_index(u, v)];
        const int a = u & 1, b = (u >> 1) & 1, c = (u >> 2) & 1;
        const int a2 = v & 1, b2 = (v >> 1) & 1, c2 = (v >> 2) & 1;
        const int A = a + a2, B = b + b2, C = c + c2;
        const R sa = R(2 * a - 1), sb = R(2 * b - 1), sc = R(2 * c - 1);
        const R sa2 = R(2 * a2 - 1), sb2 = R(2 * b2 - 1), sc2 = R(2 * c2 - 1);
        Fb.S0[B][C] += (a == a2 ? R(1) : R(-1)) * w;
        Fb.S1[A][C] += (b == b2 ? R(1) : R(-1)) * w;
        Fb.S2[A][B] += (c == c2 ? R(1) : R(-1)) * w;
        Fb.T01[a2][b][C] += sa * sb2 * w;
        Fb.T01[a][b2][C] += sb * sa2 * w;
        Fb.T02[a2][c][B] += sa * sc2 * w;
        Fb.T02[a][c2][B] += sc * sa2 * w;
        Fb.T12[b2][c][A] += sb * sc2 * w;
        Fb.T12[b][c2][A] += sc * sb2 * w;
      }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int B = 0; B < 3; ++B)
#pragma unroll
          for (int C = 0; C < 3; ++C) {
            const R w = R(LL(B, s) * LL(C, t));
            H00b[s][t] += w * Fb.S0[B][C];
            H11b[s][t] += w * Fb.S1[B][C];
            H22b[s][t] += w * Fb.S2[B][C];
          }
#pragma unroll
    for (int x = 0; x < 2; ++x)
#pragma unroll
      for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
        for (int t3 = 0; t3 < 2; ++t3) {
          R z1 = R(0), z2 = R(0);
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int C = 0; C < 3; ++C) {
              z1 += R(L1(y, t2) * LL(C, t3)) * Fb.T01[x][y][C];
              z2 += R(LL(C, t2) * L1(y, t3)) * Fb.T02[x][y][C];
            }
          Z01b[x][t2][t3] = z1;
          Z02b[x][t2][t3] = z2;
        }
#pragma unroll
    for (int t1 = 0; t1 < 2; ++t1)
#pragma unroll
      for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
        for (int t3 = 0; t3 < 2; ++t3) {
          R g = R(0);
#pragma unroll
          for (int y = 0; y < 2; ++y)
#pragma unroll
            for (int z = 0; z < 2; ++z)
#pragma unroll
              for (int A = 0; A < 3; ++A) g += R(LL(A, t1) * L1(y, t2) * L1(z, t3)) * Fb.T12[y][z][A];
          G12b[t1][t2][t3] = g;
        }
  }
  // ---- per-point geometry, reversed
  R c0[2][2][3], c1[2][2][3], c2[2][2][3];
  jac_columns<R>(ex, ey, ez, c0, c1, c2);
  R c0b[2][2][3] = {}, c1b[2][2][3] = {}, c2b[2][2][3] = {};
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
        const R idet = rcp_refined(det);
        const R f = R(0.125) * idet;
        const R g00 = H00b[q2][q3], g11 = H11b[q1][q3], g22 = H22b[q1][q2];
        R g01 = R(0), g02 = R(0);
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          g01 += R(L1(x, q1)) * Z01b[x][q2][q3];
          g02 += R(L1(x, q1)) * Z02b[x][q2][q3];
        }
        const R g12 = G12b[q1][q2][q3];
        const R d00 = r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2];
        const R d11 = r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2];
        const R d22 = r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2];
        const R d01 = r0[0] * r1[0] + r0[1] * r1[1] + r0[2] * r1[2];
        const R d02 = r0[0] * r2[0] + r0[1] * r2[1] + r0[2] * r2[2];
        const R d12 = r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2];
        const R fbar = g00 * d00 + g11 * d11 + g22 * d22 + g01 * d01 + g02 * d02 + g12 * d12;
        const R detbar = -fbar * f * idet + Dbar[q1][q2][q3] * wb;
        R rb0[3], rb1[3], rb2[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
          rb0[d] = f * (R(2) * g00 * r0[d] + g01 * r1[d] + g02 * r2[d]) + detbar * A[d];
          rb1[d] = f * (g01 * r0[d] + R(2) * g11 * r1[d] + g12 * r2[d]);
          rb2[d] = f * (g02 * r0[d] + g12 * r1[d] + R(2) * g22 * r2[d]);
        }
        R* Ab = c0b[q2][q3];
        R* Bb = c1b[q1][q3];
        R* Cb = c2b[q1][q2];
#pragma unroll
        for (int d = 0; d < 3; ++d) Ab[d] += detbar * r0[d];
        cross_acc<R>(C, rb0, Bb);  // r0 = B x C
        cross_acc<R>(rb0, B, Cb);
        cross_acc<R>(A, rb1, Cb);  // r1 = C x A
        cross_acc<R>(rb1, C, Ab);
        cross_acc<R>(B, rb2, Ab);  // r2 = A x B
        cross_acc<R>(rb2, A, Bb);
      }
  // ---- Jacobian columns -> edge vectors (transpose of the bilinear interpolation)
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        R ax = R(0), ay = R(0), az = R(0);
#pragma unroll
        for (int qs = 0; qs < 2; ++qs)
#pragma unroll
          for (int qt = 0; qt < 2; ++qt) {
            const R w = R(L1(s, qs) * L1(t, qt));
            ax += w * c0b[qs][qt][d];
            ay += w * c1b[qs][qt][d];
            az += w * c2b[qs][qt][d];
          }
        gx[s][t][d] = ax;
        gy[s][t][d] = ay;
        gz[s][t][d] = az;
      }
}

}  // namespace lor
