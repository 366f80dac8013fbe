// Integration of the 2D LOR H1 matrix on one bilinear subelement (the 2D
// variant of Section 2.2: the Q1 diffusion + mass matrix of a quadrilateral,
// 2 x 2 Gauss points), shared by the coloured and the owner-computes kernels.
#pragma once

#include "lor_h1_math.hpp"

namespace lor {

// Index of the unordered corner pair (u <= v) among the 10 pairs, u-major.
__host__ __device__ constexpr int pair_index4(int u, int v) {
  return u <= v ? 4 * u - (u * (u - 1)) / 2 + (v - u) : 4 * v - (v * (v - 1)) / 2 + (u - v);
}

// The 10 unique entries of kappa K + beta M on one bilinear quadrilateral with
// corners X[v], v = a + 2b: e_b = X(1,b) - X(0,b), f_a = X(a,1) - X(a,0)
// (formed in FP64 by the caller), J = [dx/dxi, dx/deta] at each Gauss point,
// grad phi = J^-T g_hat, 2x2 Gauss, weight 1/4.  Returns false if det J <= 0.
template <typename R>
__device__ __forceinline__ bool q1_2d_entries(const R (&e)[2][2], const R (&f)[2][2], R kap, R bet, R (&out)[10]) {
#pragma unroll
  for (int k = 0; k < 10; ++k) out[k] = R(0);
  bool ok = true;
#pragma unroll
  for (int q2 = 0; q2 < 2; ++q2)
#pragma unroll
    for (int q1 = 0; q1 < 2; ++q1) {
      // dx/dxi at eta_q2 and dx/deta at xi_q1
      R a[2], b[2];
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        a[d] = R(L1(0, q2)) * e[0][d] + R(L1(1, q2)) * e[1][d];
        b[d] = R(L1(0, q1)) * f[0][d] + R(L1(1, q1)) * f[1][d];
      }
      const R det = a[0] * b[1] - a[1] * b[0];
      ok = ok && det > R(0);
      const R idet = rcp_refined(det);
      const R wk = R(0.25) * kap * idet;
      const R wm = R(0.25) * bet * det;
      R gx[4], gy[4], ph[4];  // det * grad phi and phi at the point
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int va = v & 1, vb = v >> 1;
        const R g0 = R(va ? 1.0 : -1.0) * R(L1(vb, q2));
        const R g1 = R(L1(va, q1)) * R(vb ? 1.0 : -1.0);
        gx[v] = b[1] * g0 - a[1] * g1;
        gy[v] = -b[0] * g0 + a[0] * g1;
        ph[v] = R(L1(va, q1)) * R(L1(vb, q2));
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = u; v < 4; ++v)
          out[pair_index4(u, v)] += wk * (gx[u] * gx[v] + gy[u] * gy[v]) + wm * ph[u] * ph[v];
    }
  return ok;
}

}  // namespace lor
