// Set-up kernels of the SIPG operator: DoF and quadrature-point coordinates
// and the load-vector integral b_i = sum_K (f, phi_i)_K (Sec. 4.4 right-hand
// sides) by the operator's Gauss rule, f given at the quadrature points.
// These run once per problem, so they use one thread per output value.
// Sheared lattices map every box point p to S p.
#include "internal.h"

namespace dgmf {
namespace {

__device__ __forceinline__ void store_point(const Shear& sh, const double p[3], double* xyz, int64_t N, int64_t gid) {
  for (int d = 0; d < 3; ++d)
    xyz[d * N + gid] = sh.on ? sh.m[3 * d] * p[0] + sh.m[3 * d + 1] * p[1] + sh.m[3 * d + 2] * p[2] : p[d];
}

__global__ void k_node_coords(int n, CartGeom<double> g, Shear sh, double* __restrict__ xyz, int64_t ncells,
                              TabLayout L) {
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  const int64_t N = ncells * n3;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= N) return;
  const int64_t cell = gid / n3;
  const int loc = static_cast<int>(gid - cell * n3);
  const int idx[3] = {loc % n, (loc / n) % n, loc / (n * n)};
  const int c[3] = {static_cast<int>(cell % g.nx), static_cast<int>((cell / g.nx) % g.ny),
                    static_cast<int>(cell / (static_cast<int64_t>(g.nx) * g.ny))};
  const double* nodes = g.tab + L.nodes();
  double p[3];
  for (int d = 0; d < 3; ++d) p[d] = g.x0[d][c[d]] + g.h[d][c[d]] * nodes[idx[d]];
  store_point(sh, p, xyz, N, gid);
}

__global__ void k_qp_coords(int nq, CartGeom<double> g, Shear sh, double* __restrict__ xyz, int64_t ncells,
                            TabLayout L) {
  const int64_t q3 = static_cast<int64_t>(nq) * nq * nq;
  const int64_t M = ncells * q3;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= M) return;
  const int64_t cell = gid / q3;
  const int loc = static_cast<int>(gid - cell * q3);
  const int idx[3] = {loc % nq, (loc / nq) % nq, loc / (nq * nq)};
  const int c[3] = {static_cast<int>(cell % g.nx), static_cast<int>((cell / g.nx) % g.ny),
                    static_cast<int>(cell / (static_cast<int64_t>(g.nx) * g.ny))};
  const double* xq = g.tab + L.xq();
  double p[3];
  for (int d = 0; d < 3; ++d) p[d] = g.x0[d][c[d]] + g.h[d][c[d]] * xq[idx[d]];
  store_point(sh, p, xyz, M, gid);
}

__global__ void k_integrate(int n, int nq, CartGeom<double> g, Shear sh, const double* __restrict__ f,
                            double* __restrict__ b, int64_t ncells, TabLayout L) {
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  const int64_t q3 = static_cast<int64_t>(nq) * nq * nq;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= ncells * n3) return;
  const int64_t cell = gid / n3;
  const int loc = static_cast<int>(gid - cell * n3);
  const int i = loc % n, j = (loc / n) % n, l = loc / (n * n);
  const int c[3] = {static_cast<int>(cell % g.nx), static_cast<int>((cell / g.nx) % g.ny),
                    static_cast<int>(cell / (static_cast<int64_t>(g.nx) * g.ny))};
  const double vol = g.h[0][c[0]] * g.h[1][c[1]] * g.h[2][c[2]] * (sh.on ? fabs(sh.det) : 1.0);
  const double* S = g.tab + L.S();
  const double* w = g.tab + L.wq();
  const double* fc = f + cell * q3;
  double acc = 0.0;
  for (int qz = 0; qz < nq; ++qz) {
    const double az = w[qz] * S[qz * n + l];
    for (int qy = 0; qy < nq; ++qy) {
      const double ay = az * w[qy] * S[qy * n + j];
      double sx = 0.0;
      for (int qx = 0; qx < nq; ++qx) sx += w[qx] * S[qx * n + i] * fc[(qz * nq + qy) * nq + qx];
      acc += ay * sx;
    }
  }
  b[gid] = vol * acc;
}

// ---- iso-parametric curved cells: the box point p moves to
// x = p + amp (L_0 s_1 s_2, L_1 s_2 s_0, L_2 s_0 s_1), s_e = sin(2 pi (p_e - lo_e) / L_e),
// and a cell's map is the degree-k interpolant of x at its GLL nodes.
struct CurvBox {
  double lo[3], len[3], amp;
};

__device__ __forceinline__ double wave_of(const CurvBox& b, int e, double pe) {
  return sin(2.0 * M_PI * (pe - b.lo[e]) / b.len[e]);
}

// DoF positions: the deformation at the nodes (the interpolant equals it there)
__global__ void k_node_coords_curved(int n, CartGeom<double> g, CurvBox cb, double* __restrict__ xyz,
                                     int64_t ncells, TabLayout L) {
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  const int64_t N = ncells * n3;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= N) return;
  const int64_t cell = gid / n3;
  const int loc = static_cast<int>(gid - cell * n3);
  const int idx[3] = {loc % n, (loc / n) % n, loc / (n * n)};
  const int c[3] = {static_cast<int>(cell % g.nx), static_cast<int>((cell / g.nx) % g.ny),
                    static_cast<int>(cell / (static_cast<int64_t>(g.nx) * g.ny))};
  const double* nodes = g.tab + L.nodes();
  double p[3], sw[3];
  for (int d = 0; d < 3; ++d) {
    p[d] = g.x0[d][c[d]] + g.h[d][c[d]] * nodes[idx[d]];
    sw[d] = wave_of(cb, d, p[d]);
  }
  for (int d = 0; d < 3; ++d) xyz[d * N + gid] = p[d] + cb.amp * cb.len[d] * sw[(d + 1) % 3] * sw[(d + 2) % 3];
}

// Quadrature points: the interpolated map at the Gauss points, per direction
// sig_e(x_q) = sum_i s_e(node i) l_i(x_q) (the affine part is reproduced exactly)
__global__ void k_qp_coords_curved(int n, int nq, CartGeom<double> g, CurvBox cb, double* __restrict__ xyz,
                                   int64_t ncells, TabLayout L) {
  const int64_t q3 = static_cast<int64_t>(nq) * nq * nq;
  const int64_t M = ncells * q3;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= M) return;
  const int64_t cell = gid / q3;
  const int loc = static_cast<int>(gid - cell * q3);
  const int idx[3] = {loc % nq, (loc / nq) % nq, loc / (nq * nq)};
  const int c[3] = {static_cast<int>(cell % g.nx), static_cast<int>((cell / g.nx) % g.ny),
                    static_cast<int>(cell / (static_cast<int64_t>(g.nx) * g.ny))};
  const double* xq = g.tab + L.xq();
  const double* S = g.tab + L.S();
  const double* nodes = g.tab + L.nodes();
  double p[3], sg[3];
  for (int d = 0; d < 3; ++d) {
    const double x0 = g.x0[d][c[d]], h = g.h[d][c[d]];
    p[d] = x0 + h * xq[idx[d]];
    double acc = 0.0;
    for (int i = 0; i < n; ++i) acc = fma(wave_of(cb, d, x0 + h * nodes[i]), S[idx[d] * n + i], acc);
    sg[d] = acc;
  }
  for (int d = 0; d < 3; ++d) xyz[d * M + gid] = p[d] + cb.amp * cb.len[d] * sg[(d + 1) % 3] * sg[(d + 2) % 3];
}

// Load vector with the point weights w_q det J_q of the stored cell metric
// (cm[cell][6][q], n_q = k+1)
__global__ void k_integrate_curved(int n, const double* __restrict__ S, const double* __restrict__ cm,
                                   const double* __restrict__ f, double* __restrict__ b, int64_t ncells) {
  const int64_t n3 = static_cast<int64_t>(n) * n * n;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= ncells * n3) return;
  const int64_t cell = gid / n3;
  const int loc = static_cast<int>(gid - cell * n3);
  const int i = loc % n, j = (loc / n) % n, l = loc / (n * n);
  const double* fc = f + cell * n3;
  const double* mw = cm + cell * 7 * n3 + 6 * n3;
  double acc = 0.0;
  for (int qz = 0; qz < n; ++qz)
    for (int qy = 0; qy < n; ++qy) {
      const double a = S[qz * n + l] * S[qy * n + j];
      double sx = 0.0;
      for (int qx = 0; qx < n; ++qx) {
        const int q = (qz * n + qy) * n + qx;
        sx = fma(S[qx * n + i] * mw[q], fc[q], sx);
      }
      acc = fma(a, sx, acc);
    }
  b[gid] = acc;
}

unsigned grid_for(int64_t total) { return static_cast<unsigned>((total + 255) / 256); }

}  // namespace

dgmf_status launch_curved_coords(int n, int nq, bool quadrature, const CartGeom<double>& g, const double lo[3],
                                 const double len[3], double amp, double* xyz, int64_t ncells, hipStream_t s) {
  TabLayout L{n, nq};
  CurvBox cb{{lo[0], lo[1], lo[2]}, {len[0], len[1], len[2]}, amp};
  if (quadrature) {
    hipLaunchKernelGGL(k_qp_coords_curved, dim3(grid_for(ncells * nq * nq * nq)), dim3(256), 0, s, n, nq, g, cb, xyz,
                       ncells, L);
    DGMF_LAUNCH_CHECK("k_qp_coords_curved");
  } else {
    hipLaunchKernelGGL(k_node_coords_curved, dim3(grid_for(ncells * n * n * n)), dim3(256), 0, s, n, g, cb, xyz,
                       ncells, L);
    DGMF_LAUNCH_CHECK("k_node_coords_curved");
  }
  return DGMF_OK;
}

dgmf_status launch_integrate_curved(int n, const double* S, const double* cm, const double* f, double* b,
                                    int64_t ncells, hipStream_t s) {
  hipLaunchKernelGGL(k_integrate_curved, dim3(grid_for(ncells * n * n * n)), dim3(256), 0, s, n, S, cm, f, b, ncells);
  DGMF_LAUNCH_CHECK("k_integrate_curved");
  return DGMF_OK;
}

dgmf_status launch_node_coords(int n, const CartGeom<double>& g, const Shear& sh, double* xyz, int64_t ncells,
                               hipStream_t s) {
  TabLayout L{n, n};
  hipLaunchKernelGGL(k_node_coords, dim3(grid_for(ncells * n * n * n)), dim3(256), 0, s, n, g, sh, xyz, ncells, L);
  DGMF_LAUNCH_CHECK("k_node_coords");
  return DGMF_OK;
}

dgmf_status launch_qp_coords(int n, int nq, const CartGeom<double>& g, const Shear& sh, double* xyz,
                             int64_t ncells, hipStream_t s) {
  TabLayout L{n, nq};
  hipLaunchKernelGGL(k_qp_coords, dim3(grid_for(ncells * nq * nq * nq)), dim3(256), 0, s, nq, g, sh, xyz, ncells,
                     L);
  DGMF_LAUNCH_CHECK("k_qp_coords");
  return DGMF_OK;
}

dgmf_status launch_integrate(int n, int nq, const CartGeom<double>& g, const Shear& sh, const double* f, double* b,
                             int64_t ncells, hipStream_t s) {
  TabLayout L{n, nq};
  hipLaunchKernelGGL(k_integrate, dim3(grid_for(ncells * n * n * n)), dim3(256), 0, s, n, nq, g, sh, f, b, ncells,
                     L);
  DGMF_LAUNCH_CHECK("k_integrate");
  return DGMF_OK;
}

}  // namespace dgmf
