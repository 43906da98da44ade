// Closed-form Jacobian of the curved (iso-parametric) cells (gfx950 device code).
//
// Sec. 5 (implementation): a cell's map is the degree-k tensor interpolant, at
// its GLL nodes, of the physical positions of those nodes.  The positions
// come from the box deformation
//   x_r = p_r + amp L_r prod_{e != r} sin(2 pi (p_e - lo_e) / L_e);
// the interpolant of the affine part is exact and the product separates, so
//   x_h,r(xi) = x0_r + h_r xi_r + amp L_r prod_{e != r} sig_e(xi_e),
//   sig_e(t) = sum_i sin(2 pi (x0_e + h_e xi_i - lo_e) / L_e) l_i(t),
// and J_rd = h_r delta_rd + (r != d) amp L_r sig_d'(xi_d) sig_e(xi_e), with e
// the third direction.  A point is given per direction by the rows of l_i and
// l_i' there (a Gauss point, or an end point of the reference interval).
#pragma once
#include <hip/hip_runtime.h>

namespace dgmf {

struct CurvMap {
  const double* x0[3];   // per direction: cell origins (device)
  const double* h[3];    // per direction: cell sizes (device)
  double lo[3], len[3], amp;
  const double* nodes;   // n GLL nodes on [0, 1] (device)
};

// sig and sig' of direction e of cell coordinate ce at the point with rows val, der
template <int N>
__device__ __forceinline__ void curv_sig_at(const CurvMap& m, int e, int ce, const double* val, const double* der,
                                            double& sg, double& dsg) {
  const double x0 = m.x0[e][ce], h = m.h[e][ce];
  sg = 0.0;
  dsg = 0.0;
#pragma unroll
  for (int i = 0; i < N; ++i) {
    const double sv = sin(2.0 * M_PI * (x0 + h * m.nodes[i] - m.lo[e]) / m.len[e]);
    sg = fma(sv, val[i], sg);
    dsg = fma(sv, der[i], dsg);
  }
}

// J (row-major, J[r*3+d] = d x_r / d xi_d) of cell c at the point with per-direction rows (val[e], der[e])
template <int N>
__device__ __forceinline__ void curv_jac_at(const CurvMap& m, const int c[3], const double* const val[3],
                                            const double* const der[3], double J[9]) {
  double sg[3], dsg[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) curv_sig_at<N>(m, e, c[e], val[e], der[e], sg[e], dsg[e]);
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (r == d) {
        J[r * 3 + d] = m.h[r][c[r]];
      } else {
        const int e = 3 - r - d;
        J[r * 3 + d] = m.amp * m.len[r] * dsg[d] * sg[e];
      }
    }
}

// row e of adj(J) = det(J) J^{-1}: the cross product of columns e+1 and e+2 (cyclic)
__device__ __forceinline__ void adj_row(const double J[9], int e, double out[3]) {
  const int a = (e + 1) % 3, b = (e + 2) % 3;
  out[0] = J[1 * 3 + a] * J[2 * 3 + b] - J[2 * 3 + a] * J[1 * 3 + b];
  out[1] = J[2 * 3 + a] * J[0 * 3 + b] - J[0 * 3 + a] * J[2 * 3 + b];
  out[2] = J[0 * 3 + a] * J[1 * 3 + b] - J[1 * 3 + a] * J[0 * 3 + b];
}

}  // namespace dgmf
