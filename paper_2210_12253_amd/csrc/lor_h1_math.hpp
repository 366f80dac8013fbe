// Per-subelement integration of the LOR H1 matrix on one trilinear subelement.
//
// Section 2.2: the LOR matrix is the Q1 stiffness + mass matrix of the refined
// mesh.  On a subelement with corner coordinates X_v (v = a + 2b + 4c at the
// reference corner (a,b,c) of [0,1]^3), with 2x2x2 Gauss points q (weight 1/8):
//
//   K_uv = kappa sum_q (1/8) det J (J^-T g_u).(J^-T g_v)
//        = sum_q sum_rc  G_rc(q) g_u,r(q) g_v,c(q),   G = (kappa / 8 det J) R R^T,
//   M_uv = beta sum_q (1/8) det J phi_u phi_v,
//
// where R has the rows r_0 = J_1 x J_2, r_1 = J_2 x J_0, r_2 = J_0 x J_1 (J_c the
// columns of J, so J^-1 = R / det J).  The reference gradients are tensor
// products, g_u,0 = l_a'(xi) l_b(eta) l_c(zeta) with l_0 = 1 - t, l_1 = t, so
// l' = -1 or +1.  Every entry therefore splits into 1D pieces:
//
//   M_uv  = TM[a+a'][b+b'][c+c']
//   (r,r) terms: s_a S0[b+b'][c+c'] + s_b S1[a+a'][c+c'] + s_c S2[a+a'][b+b']
//   (r,c) terms: sig_a sig_b' T01[a'][b][c+c'] + sig_b sig_a' T01[a][b'][c+c']  (and 02, 12)
//
// with s_a = +1 if a == a' else -1, sig_a = 2a - 1, and the factor tables
//   S0[B][C]  = sum_q G00(q) LL_B(eta_q) LL_C(zeta_q)        (LL_0 = l0^2, LL_1 = l0 l1, LL_2 = l1^2)
//   T01[x][y][C] = sum_q G01(q) l_x(xi_q) l_y(eta_q) LL_C(zeta_q)   ...
//   TM[A][B][C] = sum_q (beta det J / 8) LL_A LL_B LL_C.
// They are contracted one axis at a time (sum factorisation), so a subelement
// costs about 1.3k flops instead of ~2k for the direct 8x8 quadrature.
#pragma once

#include <hip/hip_runtime.h>

namespace lor {

// l_a(t_q) at the two Gauss points t_0 = (1 - 1/sqrt3)/2, t_1 = (1 + 1/sqrt3)/2.
constexpr double kGA = 0.78867513459481288225457439025098;  // l_0(t_0) = l_1(t_1)
constexpr double kGB = 0.21132486540518711774542560974902;  // l_1(t_0) = l_0(t_1)
constexpr double kGA2 = 0.62200846792814621558800373425063;  // kGA^2
constexpr double kGB2 = 0.04465819873852045107866293241604;  // kGB^2
constexpr double kSixth = 0.16666666666666666666666666666667;  // kGA * kGB

__host__ __device__ constexpr double L1(int a, int q) { return a == q ? kGA : kGB; }
// LL_A(t_q) for A = a + a' in {0, 1, 2}
__host__ __device__ constexpr double LL(int A, int q) {
  return A == 1 ? kSixth : ((A == 0) == (q == 0) ? kGA2 : kGB2);
}

// Index of the unordered corner pair (u <= v) among the 36 pairs, u-major.
__host__ __device__ constexpr int pair_index(int u, int v) {
  return u <= v ? (u * (15 - u)) / 2 + v : (v * (15 - v)) / 2 + u;
}

// 1/x from the hardware reciprocal estimate refined by Newton steps (two in
// FP64, one in FP32): within an ulp or two, far cheaper than IEEE division.
__device__ __forceinline__ double rcp_refined(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, r, 1.0);
  r = __builtin_fma(r, e, r);
  e = __builtin_fma(-x, r, 1.0);
  return __builtin_fma(r, e, r);
}
__device__ __forceinline__ float rcp_refined(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  const float e = __builtin_fmaf(-x, r, 1.0f);
  return __builtin_fmaf(r, e, r);
}

template <typename R>
struct H1Factors {
  R S0[3][3], S1[3][3], S2[3][3];
  R T01[2][2][3], T02[2][2][3], T12[2][2][3];
  R TM[3][3][3];
};

// Edge vectors of the trilinear subelement, formed in FP64 then rounded to R:
// ex[b][c] = X(1,b,c) - X(0,b,c), ey[a][c] = X(a,1,c) - X(a,0,c),
// ez[a][b] = X(a,b,1) - X(a,b,0).
template <typename R>
__device__ __forceinline__ void h1_edges(const double (&X)[8][3], R (&ex)[2][2][3], R (&ey)[2][2][3],
                                         R (&ez)[2][2][3]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        ex[s][t][d] = static_cast<R>(X[1 + 2 * s + 4 * t][d] - X[0 + 2 * s + 4 * t][d]);
        ey[s][t][d] = static_cast<R>(X[s + 2 + 4 * t][d] - X[s + 4 * t][d]);
        ez[s][t][d] = static_cast<R>(X[s + 2 * t + 4][d] - X[s + 2 * t][d]);
      }
}

// Largest / smallest Jacobian determinant over the 8 corners (the triple
// product of the three edge vectors meeting at the corner).
template <typename R>
__device__ __forceinline__ void h1_corner_det_range(const R (&ex)[2][2][3], const R (&ey)[2][2][3],
                                                    const R (&ez)[2][2][3], R& dmin, R& dmax) {
  dmin = R(3.0e38);
  dmax = R(-3.0e38);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const R* A = ex[b][c];
        const R* B = ey[a][c];
        const R* C = ez[a][b];
        const R d = A[0] * (B[1] * C[2] - B[2] * C[1]) + A[1] * (B[2] * C[0] - B[0] * C[2]) +
                    A[2] * (B[0] * C[1] - B[1] * C[0]);
        dmin = d < dmin ? d : dmin;
        dmax = d > dmax ? d : dmax;
      }
}

// Jacobian columns at the Gauss points: J_0 = dx/dxi depends on (eta, zeta)
// only and is the bilinear interpolant of the four x-edge vectors, etc.
// c0[q2][q3], c1[q1][q3], c2[q1][q2].
template <typename R>
__device__ __forceinline__ void jac_columns(const R (&ex)[2][2][3], const R (&ey)[2][2][3], const R (&ez)[2][2][3],
                                            R (&c0)[2][2][3], R (&c1)[2][2][3], R (&c2)[2][2][3]) {
#pragma unroll
  for (int d = 0; d < 3; ++d)
#pragma unroll
    for (int qs = 0; qs < 2; ++qs) {
      const R m0x = R(L1(0, qs)) * ex[0][0][d] + R(L1(1, qs)) * ex[1][0][d];
      const R m1x = R(L1(0, qs)) * ex[0][1][d] + R(L1(1, qs)) * ex[1][1][d];
      const R m0y = R(L1(0, qs)) * ey[0][0][d] + R(L1(1, qs)) * ey[1][0][d];
      const R m1y = R(L1(0, qs)) * ey[0][1][d] + R(L1(1, qs)) * ey[1][1][d];
      const R m0z = R(L1(0, qs)) * ez[0][0][d] + R(L1(1, qs)) * ez[1][0][d];
      const R m1z = R(L1(0, qs)) * ez[0][1][d] + R(L1(1, qs)) * ez[1][1][d];
#pragma unroll
      for (int qt = 0; qt < 2; ++qt) {
        c0[qs][qt][d] = R(L1(0, qt)) * m0x + R(L1(1, qt)) * m1x;
        c1[qs][qt][d] = R(L1(0, qt)) * m0y + R(L1(1, qt)) * m1y;
        c2[qs][qt][d] = R(L1(0, qt)) * m0z + R(L1(1, qt)) * m1z;
      }
    }
}

// Contract the per-point metric values into the S and T factor tables.
//   H00[q2][q3] = sum_q1 G00,  H11[q1][q3] = sum_q2 G11,  H22[q1][q2] = sum_q3 G22,
//   Z01[x][q2][q3] = sum_q1 l_x(xi) G01,  Z02[x][q2][q3] = sum_q1 l_x(xi) G02,
//   G12q[q1][q2][q3] = G12 at every point.
template <typename R>
__device__ __forceinline__ void h1_contract_stiffness(const R (&H00)[2][2], const R (&H11)[2][2],
                                                      const R (&H22)[2][2], const R (&Z01)[2][2][2],
                                                      const R (&Z02)[2][2][2], const R (&G12q)[2][2][2],
                                                      H1Factors<R>& F) {
#pragma unroll
  for (int B = 0; B < 3; ++B) {
    R y0[2], y1[2], y2[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      y0[t] = R(LL(B, 0)) * H00[0][t] + R(LL(B, 1)) * H00[1][t];  // S0: eta -> B
      y1[t] = R(LL(B, 0)) * H11[0][t] + R(LL(B, 1)) * H11[1][t];  // S1: xi  -> B
      y2[t] = R(LL(B, 0)) * H22[0][t] + R(LL(B, 1)) * H22[1][t];  // S2: xi  -> B
    }
#pragma unroll
    for (int Cc = 0; Cc < 3; ++Cc) {
      F.S0[B][Cc] = R(LL(Cc, 0)) * y0[0] + R(LL(Cc, 1)) * y0[1];
      F.S1[B][Cc] = R(LL(Cc, 0)) * y1[0] + R(LL(Cc, 1)) * y1[1];
      F.S2[B][Cc] = R(LL(Cc, 0)) * y2[0] + R(LL(Cc, 1)) * y2[1];
    }
  }
#pragma unroll
  for (int x = 0; x < 2; ++x) {
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      // T01[x][y][C]: eta -> l_y, zeta -> LL_C
      const R t0 = R(L1(y, 0)) * Z01[x][0][0] + R(L1(y, 1)) * Z01[x][1][0];
      const R t1 = R(L1(y, 0)) * Z01[x][0][1] + R(L1(y, 1)) * Z01[x][1][1];
#pragma unroll
      for (int Cc = 0; Cc < 3; ++Cc) F.T01[x][y][Cc] = R(LL(Cc, 0)) * t0 + R(LL(Cc, 1)) * t1;
    }
#pragma unroll
    for (int z = 0; z < 2; ++z) {
      // T02[x][z][B]: zeta -> l_z, eta -> LL_B
      const R t0 = R(L1(z, 0)) * Z02[x][0][0] + R(L1(z, 1)) * Z02[x][0][1];
      const R t1 = R(L1(z, 0)) * Z02[x][1][0] + R(L1(z, 1)) * Z02[x][1][1];
#pragma unroll
      for (int B = 0; B < 3; ++B) F.T02[x][z][B] = R(LL(B, 0)) * t0 + R(LL(B, 1)) * t1;
    }
  }
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    R Z12[2][2];
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
      for (int t3 = 0; t3 < 2; ++t3)
        Z12[t2][t3] = R(LL(al, 0)) * G12q[0][t2][t3] + R(LL(al, 1)) * G12q[1][t2][t3];
#pragma unroll
    for (int y = 0; y < 2; ++y) {
      // T12[y][z][A]: xi -> LL_A, eta -> l_y, zeta -> l_z
      const R t0 = R(L1(y, 0)) * Z12[0][0] + R(L1(y, 1)) * Z12[1][0];
      const R t1 = R(L1(y, 0)) * Z12[0][1] + R(L1(y, 1)) * Z12[1][1];
#pragma unroll
      for (int z = 0; z < 2; ++z) F.T12[y][z][al] = R(L1(z, 0)) * t0 + R(L1(z, 1)) * t1;
    }
  }
}

// mass: TM[A][B][C] = sum_q D(q) LL_A(xi) LL_B(eta) LL_C(zeta)
template <typename R>
__device__ __forceinline__ void h1_contract_mass(const R (&Dq)[2][2][2], R (&TM)[3][3][3]) {
#pragma unroll
  for (int al = 0; al < 3; ++al) {
    R U[2][2];
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
      for (int t3 = 0; t3 < 2; ++t3) U[t2][t3] = R(LL(al, 0)) * Dq[0][t2][t3] + R(LL(al, 1)) * Dq[1][t2][t3];
#pragma unroll
    for (int B = 0; B < 3; ++B) {
      const R t0 = R(LL(B, 0)) * U[0][0] + R(LL(B, 1)) * U[1][0];
      const R t1 = R(LL(B, 0)) * U[0][1] + R(LL(B, 1)) * U[1][1];
#pragma unroll
      for (int Cc = 0; Cc < 3; ++Cc) TM[al][B][Cc] = R(LL(Cc, 0)) * t0 + R(LL(Cc, 1)) * t1;
    }
  }
}

// Factor tables of one subelement; returns false if det J <= 0 at a Gauss point.
template <typename R>
__device__ __forceinline__ bool h1_factors(const R (&ex)[2][2][3], const R (&ey)[2][2][3],
                                           const R (&ez)[2][2][3], R kap, R bet, H1Factors<R>& F) {
  R c0[2][2][3], c1[2][2][3], c2[2][2][3];
  jac_columns<R>(ex, ey, ez, c0, c1, c2);
  R H00[2][2] = {}, H11[2][2] = {}, H22[2][2] = {};
  R Z01[2][2][2] = {}, Z02[2][2][2] = {};
  R G12q[2][2][2], Dq[2][2][2];  // per Gauss point (q1, q2, q3): G_12 and beta det J / 8
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
        const R f = wk * rcp_refined(det);
        H00[q2][q3] += f * (r0[0] * r0[0] + r0[1] * r0[1] + r0[2] * r0[2]);
        H11[q1][q3] += f * (r1[0] * r1[0] + r1[1] * r1[1] + r1[2] * r1[2]);
        H22[q1][q2] += f * (r2[0] * r2[0] + r2[1] * r2[1] + r2[2] * r2[2]);
        const R g01 = f * (r0[0] * r1[0] + r0[1] * r1[1] + r0[2] * r1[2]);
        const R g02 = f * (r0[0] * r2[0] + r0[1] * r2[1] + r0[2] * r2[2]);
        G12q[q1][q2][q3] = f * (r1[0] * r2[0] + r1[1] * r2[1] + r1[2] * r2[2]);
        Dq[q1][q2][q3] = wb * det;
#pragma unroll
        for (int x = 0; x < 2; ++x) {
          Z01[x][q2][q3] += R(L1(x, q1)) * g01;
          Z02[x][q2][q3] += R(L1(x, q1)) * g02;
        }
      }
  h1_contract_stiffness<R>(H00, H11, H22, Z01, Z02, G12q, F);
  h1_contract_mass<R>(Dq, F.TM);
  return ok;
}

// Entry (u, v) of K + M from the factor tables.
template <typename R>
__device__ __forceinline__ R h1_entry(const H1Factors<R>& F, int u, int v) {
  const int a = u & 1, b = (u >> 1) & 1, c = (u >> 2) & 1;
  const int a2 = v & 1, b2 = (v >> 1) & 1, c2 = (v >> 2) & 1;
  const int A = a + a2, B = b + b2, C = c + c2;
  const R sa = R(2 * a - 1), sb = R(2 * b - 1), sc = R(2 * c - 1);
  const R sa2 = R(2 * a2 - 1), sb2 = R(2 * b2 - 1), sc2 = R(2 * c2 - 1);
  R val = F.TM[A][B][C];
  val += (a == a2 ? R(1) : R(-1)) * F.S0[B][C];
  val += (b == b2 ? R(1) : R(-1)) * F.S1[A][C];
  val += (c == c2 ? R(1) : R(-1)) * F.S2[A][B];
  val += sa * sb2 * F.T01[a2][b][C] + sb * sa2 * F.T01[a][b2][C];
  val += sa * sc2 * F.T02[a2][c][B] + sc * sa2 * F.T02[a][c2][B];
  val += sb * sc2 * F.T12[b2][c][A] + sc * sb2 * F.T12[b][c2][A];
  return val;
}

}  // namespace lor
