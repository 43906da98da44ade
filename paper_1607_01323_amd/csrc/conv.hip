// Convective operator with the local Lax-Friedrichs flux, the explicit
// convective substep U - dt M^{-1} C(U), and the vector-Jacobian product, on
// axis-aligned hexahedra (gfx950).
//
// C(U)_{i,a} = - sum_K (d_b phi_i, u_a u_b)_K + sum_K (phi_i, R_a)_{dK}      (Sec. 3.2, eq. convstepspat)
//   R = 1/2 (u- (u-.n) + u+ (u+.n)) + lam (u- - u+),  lam = max(|u-.n|, |u+.n|)
// evaluated at every face quadrature point; Dirichlet faces use the mirror
// state u+ = -u- (no-slip, g = 0), outflow (Neumann) faces the own state
// u+ = u-, i.e. the flux F^c(u-).n of the paper's Neumann part.  Quadrature: Q Gauss points per direction
// on cells and faces (Sec. 5 over-integration).
//
// VJP (transpose of the exact derivative of C, piecewise quadratic in U):
//   cell: g_c = -(phi, sum_b u_b d_b w_c + sum_a u_a d_c w_a)_K
//   face with L on the low side, n = +e_d, [w] = w_L - w_R:
//     g_L += phi J-^T [w],  g_R += phi J+^T [w],
//     J-^T v = 1/2 (a v + n (u-.v)) + lam v + dlam- ((u- - u+).v)
//     J+^T v = 1/2 (b v + n (u+.v)) - lam v + dlam+ ((u- - u+).v)
//     a = u-.n, b = u+.n, dlam- = sgn(a) n if |a| >= |b| else 0, dlam+ = sgn(b) n otherwise
//   Dirichlet face: g += phi (J- - J+)^T w- with u+ = -u-;
//   outflow face: g += phi (J- + J+)^T w- = phi ((u.n) w + n (u.w)) with u+ = u-.
//
// Kernel layout: one cell per workgroup.  Thread (qx, qy) owns the z-column
// of quadrature points of its (qx, qy) in registers (values, fluxes, VJP
// accumulators); sweeps along x and y are staged through LDS with one thread
// per line, or per point where that saves LDS and a barrier (FwdPlan,
// VjpPlan); faces are processed one direction (or one face) at a time and
// their lifts land on the cell's boundary node planes before a single
// coalesced store.  The substep variant applies the inverse mass block
// (Mh^{-1} along x, y and z, times 1/|det J|; Sec. 5, implementation) to the
// cell's result in LDS and writes U - dt M^{-1} C(U) in the same store, so
// C(U) never travels through HBM.
#include "curv_map.h"
#include "internal.h"

namespace dgmf {
namespace {

constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_cell(int64_t b, int64_t nblocks) {
  const int64_t q = nblocks / kXcds, rem = nblocks % kXcds;
  const int64_t x = b % kXcds, r = b / kXcds;
  return x * q + (x < rem ? x : rem) + r;
}

template <int N, int Q>
struct CShape {
  static constexpr int N2 = N * N, N3 = N2 * N, Q2 = Q * Q;
  static constexpr int THREADS = ((Q2 + 63) / 64) * 64;
};

// Unroll factor of the sweep loops that step over table rows / columns: small
// tables fit the scalar registers whole and are unrolled completely; large
// ones (n * n_q > 48) step one row or column at a time, which keeps the
// compiler from spilling table entries (six rows in flight, so the scalar
// loads of the next rows overlap the arithmetic of the current one; two and
// three measured slower at k = 5, n_q = 9, with no spills at six).
template <int N, int Q>
constexpr int kSweepUnroll = N * Q > 48 ? 6 : 16;

struct CellGeo {
  int c[3];
  double h[3], hinv[3];
};

__device__ __forceinline__ void conv_cell(const ConvGeom& g, int64_t cell, CellGeo& cg) {
  cg.c[0] = static_cast<int>(cell % g.nx);
  const int64_t r = cell / g.nx;
  cg.c[1] = static_cast<int>(r % g.ny);
  cg.c[2] = static_cast<int>(r / g.ny);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    cg.h[d] = g.h[d][cg.c[d]];
    cg.hinv[d] = g.hinv[d][cg.c[d]];
  }
}

// neighbour across face (d, s) or -1 on a Dirichlet face
__device__ __forceinline__ int64_t conv_nb(const ConvGeom& g, const CellGeo& cg, int64_t cell, int d, int s) {
  const int nd = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
  int cc = cg.c[d] + (s ? 1 : -1);
  if (cc < 0 || cc >= nd) {
    if (!g.per[d]) return -1;
    cc = cc < 0 ? nd - 1 : 0;
  }
  const int64_t stride = d == 0 ? 1 : (d == 1 ? g.nx : static_cast<int64_t>(g.nx) * g.ny);
  return cell + static_cast<int64_t>(cc - cg.c[d]) * stride;
}

// node index (l, j, i) of a face-plane entry (p1 along t1, p2 along t2) of face (d, s)
template <int N>
__device__ __forceinline__ int face_node(int d, int s, int p1, int p2) {
  const int e = s ? N - 1 : 0;
  if (d == 0) return (p2 * N + p1) * N + e;        // t1 = y, t2 = z
  if (d == 1) return (p2 * N + e) * N + p1;        // t1 = x, t2 = z
  return (e * N + p2) * N + p1;                    // t1 = x, t2 = y
}

// Interpolate NC nodal fields sIn[NC][N^3] to the quadrature z-column of
// this thread: out[a][qz].  T1 (NC*N*N*Q) and T2 (NC*N*Q*Q) are LDS scratch.
template <int N, int Q, int NC = 3>
__device__ __forceinline__ void interp3(const double* __restrict__ S, const double* sIn, double* T1, double* T2,
                                        int tid, int nthr, bool own, int qx, int qy, double (&out)[NC][Q]) {
  constexpr int N2 = N * N;
  for (int job = tid; job < NC * N2; job += nthr) {     // x: (a, l, j)
    const double* in = sIn + job * N;
    double v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = in[i];
#pragma unroll kSweepUnroll<N, Q>
    for (int q = 0; q < Q; ++q) {
      double s = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) s = fma(S[q * N + i], v[i], s);
      T1[job * Q + q] = s;
    }
  }
  __syncthreads();
  for (int job = tid; job < NC * N * Q; job += nthr) {  // y: (a, l, qx)
    const int qxx = job % Q, al = job / Q;
    double v[N];
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = T1[(al * N + j) * Q + qxx];
#pragma unroll kSweepUnroll<N, Q>
    for (int q = 0; q < Q; ++q) {
      double s = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) s = fma(S[q * N + j], v[j], s);
      T2[(al * Q + q) * Q + qxx] = s;
    }
  }
  __syncthreads();
  if (own) {                                            // z: registers, one table column per step
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
      for (int q = 0; q < Q; ++q) out[a][q] = 0.0;
#pragma unroll kSweepUnroll<N, Q>
    for (int l = 0; l < N; ++l) {
      double xv[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) xv[a] = T2[((a * N + l) * Q + qy) * Q + qx];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const double c = S[q * N + l];
#pragma unroll
        for (int a = 0; a < NC; ++a) out[a][q] = fma(c, xv[a], out[a][q]);
      }
    }
  }
}

// Interpolation of NC nodal fields sIn[NC][N^3] to the quadrature z-column
// of this thread, with the y direction taken point by point: the x sweep
// runs one line per thread into T1 ([a][l][qx][j], NC N^2 Q doubles of LDS),
// then each column thread forms its (qx, qy) values of every (a, l) from its
// own row of S (the y sweep; lanes of one qx read the same T1 entries) and
// sweeps them along z in registers.  Against interp3 this needs no second
// scratch array and one barrier less.
template <int N, int Q, int NC, int NTHR>
__device__ __forceinline__ void interp3_col(const double* __restrict__ S, const double* sIn, double* T1, int tid,
                                            bool own, int qx, int qy, double (&out)[NC][Q]) {
  constexpr int N2 = N * N;
  for (int job = tid; job < NC * N2; job += NTHR) {    // x: (a, l, j)
    const int al = job / N, j = job - al * N;
    const double* in = sIn + job * N;
    double v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = in[i];
#pragma unroll kSweepUnroll<N, Q>
    for (int q = 0; q < Q; ++q) {
      double acc = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) acc = fma(S[q * N + i], v[i], acc);
      T1[(al * Q + q) * N + j] = acc;
    }
  }
  __syncthreads();
  if (own) {
    double sy[N];
#pragma unroll
    for (int j = 0; j < N; ++j) sy[j] = S[qy * N + j];
#pragma unroll
    for (int a = 0; a < NC; ++a)
#pragma unroll
      for (int q = 0; q < Q; ++q) out[a][q] = 0.0;
#pragma unroll kSweepUnroll<N, Q>
    for (int l = 0; l < N; ++l) {
      double xv[NC];
#pragma unroll
      for (int a = 0; a < NC; ++a) {
        const double* t = T1 + ((a * N + l) * Q + qx) * N;
        double acc = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) acc = fma(sy[j], t[j], acc);
        xv[a] = acc;
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const double c = S[q * N + l];
#pragma unroll
        for (int a = 0; a < NC; ++a) out[a][q] = fma(c, xv[a], out[a][q]);
      }
    }
  }
}

// First step of face_interp with the result laid out [plane][q1][p2], for
// a second step taken point by point (each thread its own rows of S).
template <int N, int Q, int NTHR>
__device__ __forceinline__ void face_interp_t1(const double* __restrict__ S, const double* P, double* F1, int np,
                                               int tid) {
  for (int job = tid; job < np * N; job += NTHR) {     // along t1: (plane, p2)
    const int pl = job / N, p2 = job - pl * N;
    double v[N];
#pragma unroll
    for (int p = 0; p < N; ++p) v[p] = P[job * N + p];
#pragma unroll kSweepUnroll<N, Q>
    for (int q = 0; q < Q; ++q) {
      double acc = 0;
#pragma unroll
      for (int p = 0; p < N; ++p) acc = fma(S[q * N + p], v[p], acc);
      F1[(pl * Q + q) * N + p2] = acc;
    }
  }
  __syncthreads();
}

// Tangential interpolation of `np` face planes (N x N, index [p2][p1]) to
// Q x Q points ([q2][q1]); F1 (np*N*Q) scratch, F2 (np*Q*Q) result.
template <int N, int Q>
__device__ __forceinline__ void face_interp(const double* __restrict__ S, const double* P, double* F1, double* F2,
                                            int np, int tid, int nthr) {
  for (int job = tid; job < np * N; job += nthr) {     // along t1: (plane, p2)
    double v[N];
#pragma unroll
    for (int p = 0; p < N; ++p) v[p] = P[job * N + p];
#pragma unroll kSweepUnroll<N, Q>
    for (int q = 0; q < Q; ++q) {
      double s = 0;
#pragma unroll
      for (int p = 0; p < N; ++p) s = fma(S[q * N + p], v[p], s);
      F1[job * Q + q] = s;
    }
  }
  __syncthreads();
  for (int job = tid; job < np * Q; job += nthr) {     // along t2: (plane, q1)
    const int q1 = job % Q, pl = job / Q;
    double v[N];
#pragma unroll
    for (int p = 0; p < N; ++p) v[p] = F1[(pl * N + p) * Q + q1];
#pragma unroll kSweepUnroll<N, Q>
    for (int q = 0; q < Q; ++q) {
      double s = 0;
#pragma unroll
      for (int p = 0; p < N; ++p) s = fma(S[q * N + p], v[p], s);
      F2[(pl * Q + q) * Q + q1] = s;
    }
  }
  __syncthreads();
}

// Transposed tangential interpolation of `np` planes R ([q2][q1]) and
// accumulation into sO at the face nodes: sO[comp][node(p1,p2)] += sum.
// Plane pl is component pl % NC of face (d, s), s = pl / NC when s_all < 0,
// else s = s_all.
template <int N, int Q, int NC = 3>
__device__ __forceinline__ void face_lift(const double* __restrict__ S, const double* R, double* L1, double* sO,
                                          int np, int d, int s_all, int tid, int nthr) {
  constexpr int N3 = N * N * N;
  for (int job = tid; job < np * Q; job += nthr) {     // along t2: [q2][q1] -> [p2][q1]
    const int q1 = job % Q, pl = job / Q;
    double v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = R[(pl * Q + q) * Q + q1];
#pragma unroll kSweepUnroll<N, Q>
    for (int p = 0; p < N; ++p) {
      double s = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) s = fma(S[q * N + p], v[q], s);
      L1[(pl * N + p) * Q + q1] = s;
    }
  }
  __syncthreads();
  for (int job = tid; job < np * N; job += nthr) {     // along t1: [p2][q1] -> [p2][p1]
    const int p2 = job % N, pl = job / N;
    double v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = L1[(pl * N + p2) * Q + q];
    double* o = sO + (pl % NC) * N3;
    const int side = s_all < 0 ? pl / NC : s_all;
#pragma unroll kSweepUnroll<N, Q>
    for (int p1 = 0; p1 < N; ++p1) {
      double s = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) s = fma(S[q * N + p1], v[q], s);
      o[face_node<N>(d, side, p1, p2)] += s;
    }
  }
  __syncthreads();
}

// Transposed cell sweeps of one field against the reference gradients:
//   dst[i] = sg * sum_q (d phi_i/dxi_x fx + d phi_i/dxi_y fy + d phi_i/dxi_z fz)
// with fx, fy, fz the values at this thread's quadrature z-column (read by
// owning threads only): z in registers (one node l per step, the S and D
// columns of l only), then y and x through LDS.  A (3 N Q^2) and B (2 N^2 Q)
// are LDS scratch; ends with a barrier.
template <int N, int Q>
__device__ __forceinline__ void cell_lift_grad(const double* __restrict__ S, const double* __restrict__ D,
                                               const double (&fx)[Q], const double (&fy)[Q], const double (&fz)[Q],
                                               bool own, int qx, int qy, double* A, double* B, double* dst,
                                               double sg, int tid, int nthr) {
  constexpr int N2 = N * N;
  if (own) {
#pragma unroll kSweepUnroll<N, Q>
    for (int l = 0; l < N; ++l) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) {
        a0 = fma(S[qz * N + l], fx[qz], a0);
        a1 = fma(S[qz * N + l], fy[qz], a1);
        a2 = fma(D[qz * N + l], fz[qz], a2);
      }
      A[((0 * N + l) * Q + qy) * Q + qx] = a0;
      A[((1 * N + l) * Q + qy) * Q + qx] = a1;
      A[((2 * N + l) * Q + qy) * Q + qx] = a2;
    }
  }
  __syncthreads();
  for (int job = tid; job < N * Q; job += nthr) {       // y: (l, qx)
    const int qxx = job % Q, l = job / Q;
    double v1[Q], v2[Q], v3[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      v1[q] = A[((0 * N + l) * Q + q) * Q + qxx];
      v2[q] = A[((1 * N + l) * Q + q) * Q + qxx];
      v3[q] = A[((2 * N + l) * Q + q) * Q + qxx];
    }
#pragma unroll kSweepUnroll<N, Q>
    for (int j = 0; j < N; ++j) {
      double b1 = 0, b23 = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        b1 = fma(S[q * N + j], v1[q], b1);
        b23 = fma(D[q * N + j], v2[q], fma(S[q * N + j], v3[q], b23));
      }
      B[(l * N + j) * Q + qxx] = b1;
      B[N2 * Q + (l * N + j) * Q + qxx] = b23;
    }
  }
  __syncthreads();
  for (int job = tid; job < N2; job += nthr) {          // x: (l, j)
    double v1[Q], v2[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      v1[q] = B[job * Q + q];
      v2[q] = B[N2 * Q + job * Q + q];
    }
#pragma unroll kSweepUnroll<N, Q>
    for (int i = 0; i < N; ++i) {
      double s = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) s = fma(D[q * N + i], v1[q], fma(S[q * N + i], v2[q], s));
      dst[job * N + i] = sg * s;
    }
  }
  __syncthreads();
}

// Load the face plane (d, s) of cell `c` (3 components) from global memory.
template <int N>
__device__ __forceinline__ void load_plane(const double* __restrict__ U, int64_t Nd, int64_t c, int d, int s,
                                           double* P, int tid, int nthr) {
  constexpr int N2 = N * N, N3 = N2 * N;
  for (int e = tid; e < 3 * N2; e += nthr) {
    const int a = e / N2, r = e % N2;
    P[e] = U[a * Nd + c * N3 + face_node<N>(d, s, r % N, r / N)];
  }
}

// load_plane times a factor (the own cell's plane as a mirror state)
template <int N>
__device__ __forceinline__ void load_plane_scaled(const double* __restrict__ U, int64_t Nd, int64_t c, int d, int s,
                                                  double* P, double scale, int tid, int nthr) {
  constexpr int N2 = N * N, N3 = N2 * N;
  for (int e = tid; e < 3 * N2; e += nthr) {
    const int a = e / N2, r = e % N2;
    P[e] = scale * U[a * Nd + c * N3 + face_node<N>(d, s, r % N, r / N)];
  }
}

template <int N>
__device__ __forceinline__ void copy_plane(const double* sIn, int d, int s, double* P, double scale, int tid,
                                           int nthr) {
  constexpr int N2 = N * N, N3 = N2 * N;
  for (int e = tid; e < 3 * N2; e += nthr) {
    const int a = e / N2, r = e % N2;
    P[e] = scale * sIn[a * N3 + face_node<N>(d, s, r % N, r / N)];
  }
}

// ---------------------------------------------------------------- forward
// Layout choices of the forward kernel per (n, n_q): ICOL takes the y
// interpolation point by point in the column threads (interp3_col), FPT the
// face interpolation along t2 point by point with the flux; both save LDS
// (and a barrier each) for more LDS reads.  Measured on periodic boxes of
// about 7M DoF per component, FPT is faster or level at every pair and ICOL
// at all but (3, 4), (4, 5) and (6, 9).
template <int N, int Q>
struct FwdPlan {
  static constexpr bool ICOL = !((N == 3 && Q == 4) || (N == 4 && Q == 5) || (N == 6 && Q == 9));
  static constexpr bool FPT = true;
};

template <int N, int Q, bool STEP, bool CURV>
__global__ void __launch_bounds__((CShape<N, Q>::THREADS)) k_conv_fwd(const double* __restrict__ U,
                                                                    double* __restrict__ C, const ConvGeom g,
                                                                    int64_t ncells, double dt) {
  static_assert(!(STEP && CURV), "the fused substep needs the block inverse mass of affine cells");
  using SH = CShape<N, Q>;
  constexpr int N2 = SH::N2, N3 = SH::N3, Q2 = SH::Q2, Q3 = Q2 * Q;
  constexpr bool ICOL = FwdPlan<N, Q>::ICOL, FPT = FwdPlan<N, Q>::FPT;
  // The nodal values of the cell (sU) are needed only by the interpolation's
  // x sweep: they sit in the scratch behind its first stage (T1, 3 N^2 Q),
  // where the second stage (without ICOL) overwrites them; the faces read the
  // cell's own planes from global memory again.
  constexpr int XT = 3 * N2 * Q;                                            // interpolation stage 1
  constexpr int XI = XT + (ICOL ? 3 * N3 : (3 * N3 > 3 * N * Q2 ? 3 * N3 : 3 * N * Q2));
  constexpr int XC = 3 * N * Q2 + 2 * N2 * Q;                               // cell lift scratch
  constexpr int XR = XI > XC ? XI : XC;
  constexpr int XF = 12 * N2 + 12 * N * Q + (FPT ? 0 : 12 * Q2) + 6 * Q2;   // planes, traces, fluxes
  constexpr int X = XR > XF ? XR : XF;
  __shared__ double sO[3 * N3];
  __shared__ double sX[X];
  double* sU = sX + XT;
  const int tid = threadIdx.x;
  constexpr int nthr = SH::THREADS;
  const int64_t cell = xcd_cell(blockIdx.x, gridDim.x);
  if (cell >= ncells) return;
  const int64_t Nd = ncells * N3;
  const double* S = g.tab + g.S;
  const double* D = g.tab + g.D;
  const double* w = g.tab + g.w;
  CellGeo cg;
  conv_cell(g, cell, cg);
  for (int e = tid; e < 3 * N3; e += nthr) {
    const int a = e / N3, r = e % N3;
    sU[e] = U[a * Nd + cell * N3 + r];
    sO[e] = 0.0;
  }
  const bool own = tid < Q2;
  const int qx = tid % Q, qy = (tid / Q) % Q;
  // per-lane quadrature weights, read once: w_x w_y of this thread's column
  // and w_q1 w_q2 of its face points (the same points on every face)
  const double wxy = w[qx] * w[qy];
  constexpr int KF = (2 * Q2 + nthr - 1) / nthr;
  double wf[KF];
#pragma unroll
  for (int k = 0; k < KF; ++k) {
    const int pq = (tid + k * nthr) % Q2;
    wf[k] = w[pq % Q] * w[pq / Q];
  }
  __syncthreads();
  double u[3][Q];
  if constexpr (ICOL) interp3_col<N, Q, 3, nthr>(S, sU, sX, tid, own, qx, qy, u);
  else interp3<N, Q>(S, sU, sX, sX + 3 * N2 * Q, tid, nthr, own, qx, qy, u);
  __syncthreads();
  // cell term: for each a, A1 = Sz^T F_ax, A2 = Sz^T F_ay, A3 = Dz^T F_az  (z-columns in registers),
  // then B1 = Sy^T A1, B23 = Dy^T A2 + Sy^T A3, out = -(Dx^T B1 + Sx^T B23)
  const double vol = cg.h[0] * cg.h[1] * cg.h[2];
  double* A = sX;                 // 3 * N*Q*Q  ([m][l][qy][qx])
  double* B = sX + 3 * N * Q2;    // 2 * N*N*Q  ([m][l][j][qx])
  // curved cells: V_e = sum_b w adj(J)_eb u_b on this column, so that the
  // flux of component a against d/dxi_e is u_a V_e
  double V[3][CURV ? Q : 1];
  if constexpr (CURV) {
    if (own) {
      const double* Mc = g.cmet + cell * 9 * Q3 + qy * Q + qx;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz)
#pragma unroll
        for (int e = 0; e < 3; ++e)
          V[e][qz] = fma(Mc[(3 * e + 0) * Q3 + qz * Q2], u[0][qz],
                         fma(Mc[(3 * e + 1) * Q3 + qz * Q2], u[1][qz], Mc[(3 * e + 2) * Q3 + qz * Q2] * u[2][qz]));
    }
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double fx[Q], fy[Q], fz[Q];
    if (own) {
      const double wv = wxy * vol;
#pragma unroll
      for (int qz = 0; qz < Q; ++qz) {
        if constexpr (CURV) {
          fx[qz] = u[a][qz] * V[0][qz];
          fy[qz] = u[a][qz] * V[1][qz];
          fz[qz] = u[a][qz] * V[2][qz];
        } else {
          const double f = wv * w[qz] * u[a][qz];
          fx[qz] = f * u[0][qz] * cg.hinv[0];
          fy[qz] = f * u[1][qz] * cg.hinv[1];
          fz[qz] = f * u[2][qz] * cg.hinv[2];
        }
      }
    }
    cell_lift_grad<N, Q>(S, D, fx, fy, fz, own, qx, qy, A, B, sO + a * N3, -1.0, tid, nthr);
  }
  // faces, one direction at a time (the two faces of a direction touch disjoint node planes);
  // the rows of S for this thread's face points along t2 (the same on every face)
  double sr[FPT ? KF : 1][N];
  if constexpr (FPT) {
#pragma unroll
    for (int kf = 0; kf < KF; ++kf) {
      const int q2 = ((tid + kf * nthr) % Q2) / Q;
#pragma unroll
      for (int p = 0; p < N; ++p) sr[kf][p] = S[q2 * N + p];
    }
  }
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const double area = cg.h[t1] * cg.h[t2];
    double* P = sX;                   // 12 planes of N*N: [face s][side m][comp]
    double* F1 = sX + 12 * N2;        // 12 * N*Q: [plane][q1][p2] (FPT), else [plane][p2][q1]
    double* F2 = F1 + 12 * N * Q;     // 12 * Q*Q, without FPT
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      load_plane<N>(U, Nd, cell, d, s, P + (s * 2 + 0) * 3 * N2, tid, nthr);
      const int64_t nb = conv_nb(g, cg, cell, d, s);
      if (nb >= 0) load_plane<N>(U, Nd, nb, d, 1 - s, P + (s * 2 + 1) * 3 * N2, tid, nthr);
      else   // mirror u+ = -u- (no-slip) or the own state u+ = u- (outflow)
        load_plane_scaled<N>(U, Nd, cell, d, s, P + (s * 2 + 1) * 3 * N2, ((g.neu >> (2 * d + s)) & 1) ? 1.0 : -1.0,
                             tid, nthr);
    }
    __syncthreads();
    // P occupies the front of sX; interpolate along t1 into F1 (disjoint),
    // then along t2 one face point per thread, with the flux
    if constexpr (FPT) face_interp_t1<N, Q, nthr>(S, P, F1, 12, tid);
    else face_interp<N, Q>(S, P, F1, F2, 12, tid, nthr);
    double* R = FPT ? F2 : F2 + 12 * Q2;   // 6 planes of Q*Q: [face s][comp]
#pragma unroll
    for (int kf = 0; kf < KF; ++kf) {
      const int e = tid + kf * nthr;
      if (e >= 2 * Q2) continue;
      const int s = e / Q2, pq = e % Q2;
      const double wt = wf[kf] * area;
      // own state and exterior state at this face point, outward normal sign
      const double sg = s ? 1.0 : -1.0;
      const int q1 = pq % Q;
      double um[3], up[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        if constexpr (FPT) {
          const double* fo = F1 + (((s * 2 + 0) * 3 + a) * Q + q1) * N;
          const double* fe = F1 + (((s * 2 + 1) * 3 + a) * Q + q1) * N;
          double vo = 0.0, ve = 0.0;
#pragma unroll
          for (int p = 0; p < N; ++p) {
            vo = fma(sr[kf][p], fo[p], vo);
            ve = fma(sr[kf][p], fe[p], ve);
          }
          um[a] = vo;
          up[a] = ve;
        } else {
          um[a] = F2[((s * 2 + 0) * 3 + a) * Q2 + pq];
          up[a] = F2[((s * 2 + 1) * 3 + a) * Q2 + pq];
        }
      }
      double an, bn, sc;
      if constexpr (CURV) {
        // the weighted normal w dA n (along +xi_d) of this face point; R is
        // homogeneous of degree one in it
        const double* fm = g.fmet + (cell * 18 + (2 * d + s) * 3) * Q2 + pq;
        const double n0 = fm[0], n1 = fm[Q2], n2 = fm[2 * Q2];
        an = sg * fma(n0, um[0], fma(n1, um[1], n2 * um[2]));
        bn = sg * fma(n0, up[0], fma(n1, up[1], n2 * up[2]));
        sc = 1.0;
      } else {
        an = sg * um[d];
        bn = sg * up[d];
        sc = wt;
      }
      const double lam = fmax(fabs(an), fabs(bn));
#pragma unroll
      for (int a = 0; a < 3; ++a) R[(s * 3 + a) * Q2 + pq] = sc * (0.5 * (um[a] * an + up[a] * bn) + lam * (um[a] - up[a]));
    }
    __syncthreads();
    face_lift<N, Q>(S, R, F1, sO, 6, d, -1, tid, nthr);
  }
  __syncthreads();
  if constexpr (STEP) {
    // U - dt M^{-1} C(U): three 1D sweeps by Mh^{-1} (x, y, z lines of the
    // three components, in place, one line per thread) and the scale 1/|det J|
    const double* Mi = g.tab + g.Mi;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int stride = d == 0 ? 1 : (d == 1 ? N : N2);
      for (int job = tid; job < 3 * N2; job += nthr) {
        const int a = job / N2, r = job % N2;
        // line start: x lines (j, l) -> r * N; y lines (i, l) -> l N^2 + i; z lines (i, j) -> r
        const int start = d == 0 ? r * N : (d == 1 ? (r / N) * N2 + r % N : r);
        double* p = sO + a * N3 + start;
        double v[N];
#pragma unroll
        for (int m = 0; m < N; ++m) v[m] = p[m * stride];
#pragma unroll
        for (int i = 0; i < N; ++i) {
          double t = 0;
#pragma unroll
          for (int m = 0; m < N; ++m) t = fma(Mi[i * N + m], v[m], t);
          p[i * stride] = t;
        }
      }
      __syncthreads();
    }
    const double sc = -dt * cg.hinv[0] * cg.hinv[1] * cg.hinv[2];
    for (int e = tid; e < 3 * N3; e += nthr) {
      const int a = e / N3, r = e % N3;
      C[a * Nd + cell * N3 + r] = fma(sc, sO[e], U[a * Nd + cell * N3 + r]);
    }
  } else {
    for (int e = tid; e < 3 * N3; e += nthr) {
      const int a = e / N3, r = e % N3;
      C[a * Nd + cell * N3 + r] = sO[e];
    }
  }
}

// -------------------------------------------------------------------- VJP
// Layout choices of the VJP kernel per (n, n_q), as FwdPlan for the forward
// (the cell lift's scratch bounds the LDS here, so ICOL saves a barrier but
// no LDS); PAIR treats both faces of a direction in one pass (half the face
// barriers, twice the face scratch).  Measured as for the forward: ICOL and
// FPT are faster or level at every pair but (3, 4); PAIR at all but (4, 6),
// (5, 7) and (6, 8), where the larger scratch costs resident cells.
template <int N, int Q>
struct VjpPlan {
  static constexpr bool ICOL = !(N == 3 && Q == 4), FPT = !(N == 3 && Q == 4);
  static constexpr bool PAIR = FPT && !((N == 4 && Q == 6) || (N == 5 && Q == 7) || (N == 6 && Q == 8));
  // SUX keeps u's nodal values in the interpolation scratch (as the forward
  // does) and reads u's own face planes from global memory: one more resident
  // cell per CU at (6, 8); elsewhere the registers bound the occupancy and
  // the extra reads cost more
  static constexpr bool SUX = N == 6 && Q == 8;
};

// Transposed flux Jacobian of the VJP at one face point of face f = 2d + s:
// out = sc (dR/du)^T [w] on the own side, with the own and exterior traces
// of u and w (uo, ue, wo, we; we unused without neighbour).
template <bool CURV>
__device__ __forceinline__ void vjp_face_point(const ConvGeom& g, int64_t cell, int d, int s, bool hasnb, int pq,
                                               int Q2, double wt, const double (&uo)[3], const double (&ue)[3],
                                               const double (&wo)[3], const double (&we)[3], double (&out)[3]) {
  const int f = 2 * d + s;
  // normal along +xi_d: e_d on affine cells (weight wt), the weighted
  // normal w dA n of the face point on curved cells (weight 1)
  double nv[3] = {0.0, 0.0, 0.0};
  double sc;
  if constexpr (CURV) {
    const double* fm = g.fmet + (cell * 18 + f * 3) * Q2 + pq;
    nv[0] = fm[0];
    nv[1] = fm[Q2];
    nv[2] = fm[2 * Q2];
    sc = 1.0;
  } else {
    sc = wt;
  }
  // n . v for the normal above
  auto ndot = [&](const double* v) {
    if constexpr (CURV) return fma(nv[0], v[0], fma(nv[1], v[1], nv[2] * v[2]));
    else return v[d];
  };
  // res += n x
  auto nadd = [&](double* res, double x) {
    if constexpr (CURV) {
#pragma unroll
      for (int b = 0; b < 3; ++b) res[b] = fma(nv[b], x, res[b]);
    } else {
      res[d] += x;
    }
  };
  double res[3];
  if (hasnb) {
    // orient with the low cell as the minus side, n along +xi_d
    const double* um = s ? uo : ue;
    const double* up = s ? ue : uo;
    double jw[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) jw[a] = s ? (wo[a] - we[a]) : (we[a] - wo[a]);
    const double an = ndot(um), bn = ndot(up);
    const double lam = fmax(fabs(an), fabs(bn));
    const bool mact = fabs(an) >= fabs(bn);
    const double dj = (um[0] - up[0]) * jw[0] + (um[1] - up[1]) * jw[1] + (um[2] - up[2]) * jw[2];
    if (s) {   // this cell is the minus side: J-^T [w]
      const double ujw = um[0] * jw[0] + um[1] * jw[1] + um[2] * jw[2];
      const double dl = mact ? (an > 0 ? 1.0 : (an < 0 ? -1.0 : 0.0)) : 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) res[a] = 0.5 * an * jw[a] + lam * jw[a];
      nadd(res, 0.5 * ujw + dl * dj);
    } else {   // this cell is the plus side: J+^T [w]
      const double ujw = up[0] * jw[0] + up[1] * jw[1] + up[2] * jw[2];
      const double dl = mact ? 0.0 : (bn > 0 ? 1.0 : (bn < 0 ? -1.0 : 0.0));
#pragma unroll
      for (int a = 0; a < 3; ++a) res[a] = 0.5 * bn * jw[a] - lam * jw[a];
      nadd(res, 0.5 * ujw + dl * dj);
    }
  } else if ((g.neu >> f) & 1) {
    // outflow: R = u (u.n), (dR/du)^T w = (u.n) w + n (u.w), outward normal sg e_d
    const double sg = s ? 1.0 : -1.0;
    const double an = sg * ndot(uo);
    const double ujm = uo[0] * wo[0] + uo[1] * wo[1] + uo[2] * wo[2];
#pragma unroll
    for (int a = 0; a < 3; ++a) res[a] = an * wo[a];
    nadd(res, sg * ujm);
  } else {
    // Dirichlet: (J- - J+)^T w- with u+ = -u-, outward normal sg e_d
    const double sg = s ? 1.0 : -1.0;
    const double an = sg * ndot(uo), bn = sg * ndot(ue);
    const double lam = fmax(fabs(an), fabs(bn));
    const bool mact = fabs(an) >= fabs(bn);
    const double dj = (uo[0] - ue[0]) * wo[0] + (uo[1] - ue[1]) * wo[1] + (uo[2] - ue[2]) * wo[2];
    const double ujm = uo[0] * wo[0] + uo[1] * wo[1] + uo[2] * wo[2];
    const double ujp = ue[0] * wo[0] + ue[1] * wo[1] + ue[2] * wo[2];
    const double sa = an > 0 ? 1.0 : (an < 0 ? -1.0 : 0.0);
    const double sb = bn > 0 ? 1.0 : (bn < 0 ? -1.0 : 0.0);
    const double dlm = mact ? sa : 0.0, dlp = mact ? 0.0 : sb;
#pragma unroll
    for (int a = 0; a < 3; ++a) res[a] = 0.5 * (an - bn) * wo[a] + 2.0 * lam * wo[a];
    nadd(res, sg * (0.5 * (ujm - ujp) + (dlm - dlp) * dj));
  }
#pragma unroll
  for (int a = 0; a < 3; ++a) out[a] = sc * res[a];
}

template <int N, int Q, bool CURV>
__global__ void __launch_bounds__((CShape<N, Q>::THREADS)) k_conv_vjp(const double* __restrict__ U,
                                                                    const double* __restrict__ W,
                                                                    double* __restrict__ G, const ConvGeom g,
                                                                    int64_t ncells) {
  using SH = CShape<N, Q>;
  constexpr int N2 = SH::N2, N3 = SH::N3, Q2 = SH::Q2, Q3 = Q2 * Q;
  constexpr bool ICOL = VjpPlan<N, Q>::ICOL, FPT = VjpPlan<N, Q>::FPT, PAIR = VjpPlan<N, Q>::PAIR,
                 SUX = VjpPlan<N, Q>::SUX;
  // with SUX, the cell's nodal values of u sit in the interpolation scratch
  // behind its first stage (as in the forward)
  constexpr int XT = 3 * N2 * Q;                                              // interpolation stage 1
  constexpr int XS = ICOL ? 0 : 3 * N * Q2;                                   // interpolation stage 2
  constexpr int XI = XT + (SUX ? (3 * N3 > XS ? 3 * N3 : XS) : XS);
  constexpr int XD = 2 * N2 * Q + 3 * N * Q2;                                 // gradient scratch
  constexpr int XL = 3 * N * Q2 + 3 * N2 * Q;                                 // cell lift scratch
  constexpr int XF = PAIR ? 24 * N2 + 24 * N * Q + 6 * Q2                      // two faces: 24 planes + fluxes
                          : 12 * N2 + 12 * N * Q + (FPT ? 0 : 12 * Q2) + 3 * Q2;   // one face: 12 planes + fluxes
  constexpr int XID = XI > XD ? XI : XD, XLF = XL > XF ? XL : XF;
  constexpr int X = XID > XLF ? XID : XLF;
  __shared__ double sW[3 * N3];
  __shared__ double sO[3 * N3];
  __shared__ double sX[X];
  __shared__ double sUa[SUX ? 1 : 3 * N3];
  double* sU = SUX ? sX + XT : sUa;
  const int tid = threadIdx.x;
  constexpr int nthr = SH::THREADS;
  const int64_t cell = xcd_cell(blockIdx.x, gridDim.x);
  if (cell >= ncells) return;
  const int64_t Nd = ncells * N3;
  const double* S = g.tab + g.S;
  const double* D = g.tab + g.D;
  const double* w = g.tab + g.w;
  CellGeo cg;
  conv_cell(g, cell, cg);
  for (int e = tid; e < 3 * N3; e += nthr) {
    const int a = e / N3, r = e % N3;
    sU[e] = U[a * Nd + cell * N3 + r];
    sW[e] = W[a * Nd + cell * N3 + r];
    sO[e] = 0.0;
  }
  const bool own = tid < Q2;
  const int qx = tid % Q, qy = (tid / Q) % Q;
  // w_x w_y of this thread's column, which is also the weight of its face
  // point (at most one per face: the workgroup has at least Q^2 threads)
  static_assert(nthr >= Q2, "one face point per thread");
  const double wxy = w[qx] * w[qy];
  __syncthreads();
  double u[3][Q];
  if constexpr (ICOL) interp3_col<N, Q, 3, nthr>(S, sU, sX, tid, own, qx, qy, u);
  else interp3<N, Q>(S, sU, sX, sX + 3 * N2 * Q, tid, nthr, own, qx, qy, u);
  __syncthreads();
  double t[3][Q];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int q = 0; q < Q; ++q) t[a][q] = 0.0;
  double* T1 = sX;                  // [Sx w | Dx w] : 2 * N*N*Q, layout [m][l][j][qx]
  double* T2 = sX + 2 * N2 * Q;     // [SySx | DySx | SyDx] : 3 * N*Q*Q, layout [m][l][qy][qx]
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const double* wa = sW + a * N3;
    for (int job = tid; job < N2; job += nthr) {        // x: (l, j)
      double v[N];
#pragma unroll
      for (int i = 0; i < N; ++i) v[i] = wa[job * N + i];
#pragma unroll kSweepUnroll<N, Q>
      for (int q = 0; q < Q; ++q) {
        double s0 = 0, s1 = 0;
#pragma unroll
        for (int i = 0; i < N; ++i) {
          s0 = fma(S[q * N + i], v[i], s0);
          s1 = fma(D[q * N + i], v[i], s1);
        }
        T1[job * Q + q] = s0;
        T1[N2 * Q + job * Q + q] = s1;
      }
    }
    __syncthreads();
    for (int job = tid; job < N * Q; job += nthr) {     // y: (l, qx)
      const int qxx = job % Q, l = job / Q;
      double v0[N], v1[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        v0[j] = T1[(l * N + j) * Q + qxx];
        v1[j] = T1[N2 * Q + (l * N + j) * Q + qxx];
      }
#pragma unroll kSweepUnroll<N, Q>
      for (int q = 0; q < Q; ++q) {
        double ss = 0, ds = 0, sd = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          ss = fma(S[q * N + j], v0[j], ss);
          ds = fma(D[q * N + j], v0[j], ds);
          sd = fma(S[q * N + j], v1[j], sd);
        }
        T2[((0 * N + l) * Q + q) * Q + qxx] = ss;
        T2[((1 * N + l) * Q + q) * Q + qxx] = ds;
        T2[((2 * N + l) * Q + q) * Q + qxx] = sd;
      }
    }
    __syncthreads();
    if (own) {                                          // z: gradient of w_a on this column
      double gzq[Q], gyq[Q], gxq[Q];
#pragma unroll
      for (int q = 0; q < Q; ++q) gzq[q] = gyq[q] = gxq[q] = 0.0;
      // one node l per step: the S and D columns of l only
#pragma unroll kSweepUnroll<N, Q>
      for (int l = 0; l < N; ++l) {
        const double v0 = T2[((0 * N + l) * Q + qy) * Q + qx];
        const double v1 = T2[((1 * N + l) * Q + qy) * Q + qx];
        const double v2 = T2[((2 * N + l) * Q + qy) * Q + qx];
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          gzq[q] = fma(D[q * N + l], v0, gzq[q]);
          gyq[q] = fma(S[q * N + l], v1, gyq[q]);
          gxq[q] = fma(S[q * N + l], v2, gxq[q]);
        }
      }
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        double gz = gzq[q], gy = gyq[q], gx = gxq[q];
        if constexpr (CURV) {
          // w det J times the physical gradient: sum_e w adj(J)_eb dw/dxi_e
          const double* Mq = g.cmet + cell * 9 * Q3 + q * Q2 + qy * Q + qx;
          const double r0 = gx, r1 = gy, r2 = gz;
          gx = fma(Mq[0 * Q3], r0, fma(Mq[3 * Q3], r1, Mq[6 * Q3] * r2));
          gy = fma(Mq[1 * Q3], r0, fma(Mq[4 * Q3], r1, Mq[7 * Q3] * r2));
          gz = fma(Mq[2 * Q3], r0, fma(Mq[5 * Q3], r1, Mq[8 * Q3] * r2));
        } else {
          gx *= cg.hinv[0];
          gy *= cg.hinv[1];
          gz *= cg.hinv[2];
        }
        // t_a += u . grad w_a ;  t_b += u_a d_b w_a
        t[a][q] = fma(u[0][q], gx, fma(u[1][q], gy, fma(u[2][q], gz, t[a][q])));
        t[0][q] = fma(u[a][q], gx, t[0][q]);
        t[1][q] = fma(u[a][q], gy, t[1][q]);
        t[2][q] = fma(u[a][q], gz, t[2][q]);
      }
    }
    __syncthreads();
  }
  // g_c = -(S x S x S)^T (w vol t_c): z in registers, then y and x through LDS
  const double vol = cg.h[0] * cg.h[1] * cg.h[2];
  double* Z = sX;                   // 3 * N*Q*Q  [c][l][qy][qx]
  double* Y = sX + 3 * N * Q2;      // 3 * N*N*Q  [c][l][j][qx]
  if (own) {
    if constexpr (!CURV) {   // curved cells carry w det J in the metric already
      const double wv = wxy * vol;
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int q = 0; q < Q; ++q) t[c][q] *= wv * w[q];
    }
    // one node l per step: the S column of l only
#pragma unroll kSweepUnroll<N, Q>
    for (int l = 0; l < N; ++l) {
      double a0 = 0.0, a1 = 0.0, a2 = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const double c = S[q * N + l];
        a0 = fma(c, t[0][q], a0);
        a1 = fma(c, t[1][q], a1);
        a2 = fma(c, t[2][q], a2);
      }
      Z[((0 * N + l) * Q + qy) * Q + qx] = a0;
      Z[((1 * N + l) * Q + qy) * Q + qx] = a1;
      Z[((2 * N + l) * Q + qy) * Q + qx] = a2;
    }
  }
  __syncthreads();
  for (int job = tid; job < 3 * N * Q; job += nthr) {   // y: (c, l, qx)
    const int qxx = job % Q, cl = job / Q;
    double v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = Z[(cl * Q + q) * Q + qxx];
#pragma unroll kSweepUnroll<N, Q>
    for (int j = 0; j < N; ++j) {
      double s = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) s = fma(S[q * N + j], v[q], s);
      Y[(cl * N + j) * Q + qxx] = s;
    }
  }
  __syncthreads();
  for (int job = tid; job < 3 * N2; job += nthr) {      // x: (c, l, j)
    double v[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) v[q] = Y[job * Q + q];
#pragma unroll kSweepUnroll<N, Q>
    for (int i = 0; i < N; ++i) {
      double s = 0;
#pragma unroll
      for (int q = 0; q < Q; ++q) s = fma(S[q * N + i], v[q], s);
      sO[job * N + i] = -s;
    }
  }
  __syncthreads();
  // row qy of S, for the face points of this thread along t2 (FPT)
  double sy[N];
#pragma unroll
  for (int p = 0; p < N; ++p) sy[p] = S[qy * N + p];
  if constexpr (PAIR) {
    // faces, both of a direction at once: 24 planes = [side s][u own, u ext, w own, w ext][component]
    constexpr int KV = (2 * Q2 + nthr - 1) / nthr;
    double wv[KV], sv[KV][N];   // weights and rows of S along t2 of this thread's face points
#pragma unroll
    for (int k2 = 0; k2 < KV; ++k2) {
      const int pq = (tid + k2 * nthr) % Q2;
      wv[k2] = w[pq % Q] * w[pq / Q];
#pragma unroll
      for (int p = 0; p < N; ++p) sv[k2][p] = S[(pq / Q) * N + p];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
      const double area = cg.h[t1] * cg.h[t2];
      double* P = sX;
      double* F1 = sX + 24 * N2;        // 24 * N*Q, [plane][q1][p2]
      double* R = F1 + 24 * N * Q;      // 6 planes of Q*Q: [side s][component]
      const int64_t nb0 = conv_nb(g, cg, cell, d, 0), nb1 = conv_nb(g, cg, cell, d, 1);
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        double* Ps = P + s * 12 * N2;
        const int64_t nb = s ? nb1 : nb0;
        if constexpr (SUX) load_plane<N>(U, Nd, cell, d, s, Ps + 0 * 3 * N2, tid, nthr);
        else copy_plane<N>(sU, d, s, Ps + 0 * 3 * N2, 1.0, tid, nthr);
        copy_plane<N>(sW, d, s, Ps + 2 * 3 * N2, 1.0, tid, nthr);
        if (nb >= 0) {
          load_plane<N>(U, Nd, nb, d, 1 - s, Ps + 1 * 3 * N2, tid, nthr);
          load_plane<N>(W, Nd, nb, d, 1 - s, Ps + 3 * 3 * N2, tid, nthr);
        } else {
          if constexpr (SUX) load_plane_scaled<N>(U, Nd, cell, d, s, Ps + 1 * 3 * N2, -1.0, tid, nthr);
          else copy_plane<N>(sU, d, s, Ps + 1 * 3 * N2, -1.0, tid, nthr);
          copy_plane<N>(sW, d, s, Ps + 3 * 3 * N2, 0.0, tid, nthr);   // not used
        }
      }
      __syncthreads();
      face_interp_t1<N, Q, nthr>(S, P, F1, 24, tid);
#pragma unroll
      for (int k2 = 0; k2 < KV; ++k2) {
        const int e = tid + k2 * nthr;
        if (e >= 2 * Q2) continue;
        const int s = e / Q2, pq = e - s * Q2, q1 = pq % Q;
        const bool hb = (s ? nb1 : nb0) >= 0;
        auto along_t2 = [&](int pl) {
          const double* f = F1 + ((s * 12 + pl) * Q + q1) * N;
          double acc = 0.0;
#pragma unroll
          for (int p = 0; p < N; ++p) acc = fma(sv[k2][p], f[p], acc);
          return acc;
        };
        double uo[3], ue[3], wo[3], we[3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          uo[a] = along_t2(0 * 3 + a);
          ue[a] = along_t2(1 * 3 + a);
          wo[a] = along_t2(2 * 3 + a);
          we[a] = hb ? along_t2(3 * 3 + a) : 0.0;
        }
        double rr[3];
        vjp_face_point<CURV>(g, cell, d, s, hb, pq, Q2, wv[k2] * area, uo, ue, wo, we, rr);
#pragma unroll
        for (int a = 0; a < 3; ++a) R[(s * 3 + a) * Q2 + pq] = rr[a];
      }
      __syncthreads();
      face_lift<N, Q>(S, R, F1, sO, 6, d, -1, tid, nthr);
    }
  } else {
  // faces, one at a time: 12 planes = [u own, u ext, w own, w ext] x 3 components
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1, s = f & 1;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const double area = cg.h[t1] * cg.h[t2];
    double* P = sX;
    double* F1 = sX + 12 * N2;        // 12 * N*Q: [plane][q1][p2] (FPT), else [plane][p2][q1]
    double* F2 = F1 + 12 * N * Q;     // 12 * Q*Q, without FPT
    const int64_t nb = conv_nb(g, cg, cell, d, s);
    if constexpr (SUX) load_plane<N>(U, Nd, cell, d, s, P + 0 * 3 * N2, tid, nthr);
    else copy_plane<N>(sU, d, s, P + 0 * 3 * N2, 1.0, tid, nthr);
    copy_plane<N>(sW, d, s, P + 2 * 3 * N2, 1.0, tid, nthr);
    if (nb >= 0) {
      load_plane<N>(U, Nd, nb, d, 1 - s, P + 1 * 3 * N2, tid, nthr);
      load_plane<N>(W, Nd, nb, d, 1 - s, P + 3 * 3 * N2, tid, nthr);
    } else {
      if constexpr (SUX) load_plane_scaled<N>(U, Nd, cell, d, s, P + 1 * 3 * N2, -1.0, tid, nthr);
      else copy_plane<N>(sU, d, s, P + 1 * 3 * N2, -1.0, tid, nthr);
    }
    __syncthreads();
    if constexpr (FPT) face_interp_t1<N, Q, nthr>(S, P, F1, nb >= 0 ? 12 : 9, tid);
    else face_interp<N, Q>(S, P, F1, F2, nb >= 0 ? 12 : 9, tid, nthr);
    double* R = FPT ? F2 : F2 + 12 * Q2;   // 3 planes of Q*Q
    if (own) {
      const int pq = tid;
      const double wt = wxy * area;
      double uo[3], ue[3], wo[3], we[3];
      if constexpr (FPT) {
        // along t2 at this point: row qy of S (t1 = qx, t2 = qy on the
        // face's point grid pq = q2 Q + q1)
        auto along_t2 = [&](int pl) {
          const double* f = F1 + (pl * Q + qx) * N;
          double acc = 0.0;
#pragma unroll
          for (int p = 0; p < N; ++p) acc = fma(sy[p], f[p], acc);
          return acc;
        };
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          uo[a] = along_t2(0 * 3 + a);
          ue[a] = along_t2(1 * 3 + a);
          wo[a] = along_t2(2 * 3 + a);
          we[a] = nb >= 0 ? along_t2(3 * 3 + a) : 0.0;
        }
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          uo[a] = F2[(0 * 3 + a) * Q2 + pq];
          ue[a] = F2[(1 * 3 + a) * Q2 + pq];
          wo[a] = F2[(2 * 3 + a) * Q2 + pq];
          we[a] = nb >= 0 ? F2[(3 * 3 + a) * Q2 + pq] : 0.0;
        }
      }
      double rr[3];
      vjp_face_point<CURV>(g, cell, d, s, nb >= 0, pq, Q2, wt, uo, ue, wo, we, rr);
#pragma unroll
      for (int a = 0; a < 3; ++a) R[a * Q2 + pq] = rr[a];
    }
    __syncthreads();
    face_lift<N, Q>(S, R, F1, sO, 3, d, s, tid, nthr);
  }
  }
  __syncthreads();
  for (int e = tid; e < 3 * N3; e += nthr) {
    const int a = e / N3, r = e % N3;
    G[a * Nd + cell * N3 + r] = sO[e];
  }
}

// ------------------------------------------ V3c divergence / gradient, curved
// The divergence A (eq. av3) and gradient B (eq. bv3) of variant V3c on
// curved cells, through the quadrature points with the per-point metric of
// the fill below (n_q = k+1, the operators' own rule):
//   (A u)_i     = sum_q sum_e dphi_i/dxi_e (w adj(J) u)_e   - sum_F sum_p phi_i {{u}} . nu
//   (B p)_{i,a} = sum_q sum_e dphi_i/dxi_e (w adj(J))_{ea} p - sum_F sum_p phi_i {{p}} nu_a
// nu the weighted outward normal, {{.}} the central average inside and the
// own trace on boundary faces (Dirichlet and Neumann alike, Sec. 3.1).  One
// cell per workgroup, the layout of the convective kernels.
template <int N, int Q>
__global__ void __launch_bounds__((CShape<N, Q>::THREADS)) k_curv_div(const double* __restrict__ U,
                                                                    double* __restrict__ out, const ConvGeom g,
                                                                    int64_t ncells) {
  using SH = CShape<N, Q>;
  constexpr int N2 = SH::N2, N3 = SH::N3, Q2 = SH::Q2, Q3 = Q2 * Q;
  constexpr int XR = (3 * N2 * Q + 3 * N * Q2) > (3 * N * Q2 + 2 * N2 * Q) ? (3 * N2 * Q + 3 * N * Q2)
                                                                              : (3 * N * Q2 + 2 * N2 * Q);
  constexpr int XF = 12 * N2 + 12 * N * Q + 12 * Q2 + 2 * Q2;   // planes [s][own | ext][comp], stage, traces, flux
  constexpr int X = XR > XF ? XR : XF;
  __shared__ double sU[3 * N3];
  __shared__ double sO[N3];
  __shared__ double sX[X];
  const int tid = threadIdx.x;
  constexpr int nthr = SH::THREADS;
  const int64_t cell = xcd_cell(blockIdx.x, gridDim.x);
  if (cell >= ncells) return;
  const int64_t Nd = ncells * N3;
  const double* S = g.tab + g.S;
  const double* D = g.tab + g.D;
  CellGeo cg;
  conv_cell(g, cell, cg);
  for (int e = tid; e < 3 * N3; e += nthr) {
    const int a = e / N3, r = e % N3;
    sU[e] = U[a * Nd + cell * N3 + r];
  }
  __syncthreads();
  const bool own = tid < Q2;
  const int qx = tid % Q, qy = (tid / Q) % Q;
  double u[3][Q];
  interp3<N, Q>(S, sU, sX, sX + 3 * N2 * Q, tid, nthr, own, qx, qy, u);
  __syncthreads();
  double fe[3][Q];
  if (own) {
    const double* Mc = g.cmet + cell * 9 * Q3 + qy * Q + qx;
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
      for (int e = 0; e < 3; ++e)
        fe[e][q] = fma(Mc[(3 * e + 0) * Q3 + q * Q2], u[0][q],
                       fma(Mc[(3 * e + 1) * Q3 + q * Q2], u[1][q], Mc[(3 * e + 2) * Q3 + q * Q2] * u[2][q]));
  }
  cell_lift_grad<N, Q>(S, D, fe[0], fe[1], fe[2], own, qx, qy, sX, sX + 3 * N * Q2, sO, 1.0, tid, nthr);
  // faces, both of a direction at once (they touch disjoint node planes):
  // out -= phi ({{u}} . nu_out)
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double* P = sX;                   // 12 planes of N*N: [s][own | ext][comp]
    double* F1 = sX + 12 * N2;
    double* F2 = F1 + 12 * N * Q;
    double* R = F2 + 12 * Q2;         // 2 planes: [s]
    bool in0 = false, in1 = false;   // the face (d, s) has a neighbour
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int64_t nb = conv_nb(g, cg, cell, d, s);
      (s ? in1 : in0) = nb >= 0;
      copy_plane<N>(sU, d, s, P + (s * 2 + 0) * 3 * N2, 1.0, tid, nthr);
      if (nb >= 0) load_plane<N>(U, Nd, nb, d, 1 - s, P + (s * 2 + 1) * 3 * N2, tid, nthr);
      else copy_plane<N>(sU, d, s, P + (s * 2 + 1) * 3 * N2, 1.0, tid, nthr);   // own trace on boundary faces
    }
    __syncthreads();
    face_interp<N, Q>(S, P, F1, F2, 12, tid, nthr);
    for (int e = tid; e < 2 * Q2; e += nthr) {
      const int s = e / Q2, pq = e % Q2;
      const double* fm = g.fmet + (cell * 18 + (2 * d + s) * 3) * Q2 + pq;
      double acc = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double uo = F2[((s * 2 + 0) * 3 + a) * Q2 + pq], ue = F2[((s * 2 + 1) * 3 + a) * Q2 + pq];
        acc = fma(fm[a * Q2], (s ? in1 : in0) ? 0.5 * (uo + ue) : uo, acc);
      }
      R[s * Q2 + pq] = (s ? -1.0 : 1.0) * acc;   // minus the outward sign
    }
    __syncthreads();
    face_lift<N, Q, 1>(S, R, F1, sO, 2, d, -1, tid, nthr);
  }
  for (int e = tid; e < N3; e += nthr) out[cell * N3 + e] = sO[e];
}

template <int N, int Q>
__global__ void __launch_bounds__((CShape<N, Q>::THREADS)) k_curv_grad(const double* __restrict__ Pin,
                                                                     double* __restrict__ out, const ConvGeom g,
                                                                     int64_t ncells) {
  using SH = CShape<N, Q>;
  constexpr int N2 = SH::N2, N3 = SH::N3, Q2 = SH::Q2, Q3 = Q2 * Q;
  constexpr int XR = (N2 * Q + N * Q2) > (3 * N * Q2 + 2 * N2 * Q) ? (N2 * Q + N * Q2) : (3 * N * Q2 + 2 * N2 * Q);
  constexpr int XF = 4 * N2 + 4 * N * Q + 4 * Q2 + 6 * Q2;   // planes [s][own | ext], stage, traces, fluxes
  constexpr int X = XR > XF ? XR : XF;
  __shared__ double sP[N3];
  __shared__ double sO[3 * N3];
  __shared__ double sX[X];
  const int tid = threadIdx.x;
  constexpr int nthr = SH::THREADS;
  const int64_t cell = xcd_cell(blockIdx.x, gridDim.x);
  if (cell >= ncells) return;
  const int64_t Nd = ncells * N3;
  const double* S = g.tab + g.S;
  const double* D = g.tab + g.D;
  CellGeo cg;
  conv_cell(g, cell, cg);
  for (int e = tid; e < N3; e += nthr) sP[e] = Pin[cell * N3 + e];
  __syncthreads();
  const bool own = tid < Q2;
  const int qx = tid % Q, qy = (tid / Q) % Q;
  double p[1][Q];
  interp3<N, Q, 1>(S, sP, sX, sX + N2 * Q, tid, nthr, own, qx, qy, p);
  __syncthreads();
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double fe[3][Q];
    if (own) {
      const double* Mc = g.cmet + cell * 9 * Q3 + qy * Q + qx;
#pragma unroll
      for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int e = 0; e < 3; ++e) fe[e][q] = Mc[(3 * e + a) * Q3 + q * Q2] * p[0][q];
    }
    cell_lift_grad<N, Q>(S, D, fe[0], fe[1], fe[2], own, qx, qy, sX, sX + 3 * N * Q2, sO + a * N3, 1.0, tid,
                         nthr);
  }
  // faces, both of a direction at once: out_a -= phi {{p}} nu_out,a
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    double* P = sX;                   // 4 planes of N*N: [s][own | ext]
    double* F1 = sX + 4 * N2;
    double* F2 = F1 + 4 * N * Q;
    double* R = F2 + 4 * Q2;          // 6 planes: [s][comp]
    bool in0 = false, in1 = false;   // the face (d, s) has a neighbour
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      const int64_t nb = conv_nb(g, cg, cell, d, s);
      (s ? in1 : in0) = nb >= 0;
      for (int e = tid; e < N2; e += nthr) {
        const double own = sP[face_node<N>(d, s, e % N, e / N)];
        P[(s * 2 + 0) * N2 + e] = own;
        P[(s * 2 + 1) * N2 + e] = nb >= 0 ? Pin[nb * N3 + face_node<N>(d, 1 - s, e % N, e / N)] : own;
      }
    }
    __syncthreads();
    face_interp<N, Q>(S, P, F1, F2, 4, tid, nthr);
    for (int e = tid; e < 2 * Q2; e += nthr) {
      const int s = e / Q2, pq = e % Q2;
      const double* fm = g.fmet + (cell * 18 + (2 * d + s) * 3) * Q2 + pq;
      const double po = F2[(s * 2 + 0) * Q2 + pq], pe = F2[(s * 2 + 1) * Q2 + pq];
      const double pa = (s ? -1.0 : 1.0) * ((s ? in1 : in0) ? 0.5 * (po + pe) : po);   // minus the outward sign
#pragma unroll
      for (int a = 0; a < 3; ++a) R[(s * 3 + a) * Q2 + pq] = fm[a * Q2] * pa;
    }
    __syncthreads();
    face_lift<N, Q>(S, R, F1, sO, 6, d, -1, tid, nthr);
  }
  for (int e = tid; e < 3 * N3; e += nthr) {
    const int a = e / N3, r = e % N3;
    out[a * Nd + cell * N3 + r] = sO[e];
  }
}

// ------------------------------- V3c div-div penalty and projection, curved
// Cell-local forms of eqs. tauD, div-div and project (tau_C = 0) on curved
// cells with k+1 Gauss points per direction (n_q = n, so the point grid has
// the node grid's size): one 64-lane workgroup per cell, every vector in LDS,
// 1D operators applied line by line (one line per lane).  Per point: G =
// w sgn(det J) adj(J) from the fill below and w |det J| from the SIPG metric.
//   (M u)_{i,a}  = sum_q phi_i w|det J| u_a
//   (D u)_{i,a}  = sum_q sum_e dphi_i/dxi_e G_ea s,   s = (sum_{e,b} G_eb du_b/dxi_e) / (w |det J|)
// (w|det J| div v div u at every point), and M^{-1} = S^{-1} (x) 3 diag(1/(w|det J|)) S^{-T} (x) 3.

// Pointers whose address space the compiler could not infer through the
// per-cell structure below (flat loads, which also stall the LDS waits):
// tables read with wavefront-uniform indices go through the constant address
// space (scalar loads), per-point data through global memory.
using ctab_ptr = const __attribute__((address_space(4))) double*;
using gmem_ptr = const __attribute__((address_space(1))) double*;

// x <- A x along direction d on nb consecutive n^3 blocks (TR: A^T x); A row-major n x n
template <int N, bool TR, typename PT>
__device__ __forceinline__ void qsweep(PT A, double* buf, int nb, int d, int tid, int nthr) {
  constexpr int N2 = N * N, N3 = N2 * N;
  const int stride = d == 0 ? 1 : (d == 1 ? N : N2);
  for (int job = tid; job < nb * N2; job += nthr) {
    const int b = job / N2, r = job % N2;
    const int start = d == 0 ? r * N : (d == 1 ? (r / N) * N2 + r % N : r);
    double* p = buf + b * N3 + start;
    double v[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = p[m * stride];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double t = 0.0;
#pragma unroll
      for (int m = 0; m < N; ++m) t = fma(TR ? A[m * N + i] : A[i * N + m], v[m], t);
      p[i * stride] = t;
    }
  }
}

// sum over the 64 lanes of the (single-wavefront) workgroup; every lane gets the total
__device__ __forceinline__ double wave_total(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

struct CurvCell {
  ctab_ptr S;      // n x n: S[q][i] = l_i(x_q)
  ctab_ptr D;      // n x n: l_i'(x_q)
  ctab_ptr Si;     // n x n: S^{-1}
  gmem_ptr G;      // 9 n^3 of this cell
  gmem_ptr wd;     // n^3 of this cell: w |det J|
};

// out = (M + tau D) u on one cell; u, out [3][n^3]; W: 8 n^3 scratch
template <int N>
__device__ __forceinline__ void curv_mdd(const CurvCell& c, double tau, const double* u, double* out, double* W,
                                         int tid, int nthr) {
  constexpr int N3 = N * N * N;
  double* X1 = W;
  double* X2 = W + N3;
  double* A = W + 2 * N3;
  double* B = W + 3 * N3;
  double* V = W + 4 * N3;       // 3 blocks: point values of the components
  double* s = W + 7 * N3;
  for (int e = tid; e < N3; e += nthr) s[e] = 0.0;
  for (int a = 0; a < 3; ++a) {
    for (int e = tid; e < N3; e += nthr) X1[e] = X2[e] = u[a * N3 + e];
    __syncthreads();
    qsweep<N, false>(c.S, X1, 1, 0, tid, nthr);
    qsweep<N, false>(c.D, X2, 1, 0, tid, nthr);
    __syncthreads();
    for (int e = tid; e < N3; e += nthr) A[e] = B[e] = X1[e];
    __syncthreads();
    qsweep<N, false>(c.S, A, 1, 1, tid, nthr);   // SySx
    qsweep<N, false>(c.D, B, 1, 1, tid, nthr);   // DySx
    qsweep<N, false>(c.S, X2, 1, 1, tid, nthr);  // SyDx
    __syncthreads();
    for (int e = tid; e < N3; e += nthr) X1[e] = A[e];
    __syncthreads();
    qsweep<N, false>(c.S, X1, 1, 2, tid, nthr);  // value
    qsweep<N, false>(c.D, A, 1, 2, tid, nthr);   // d/dxi_z
    qsweep<N, false>(c.S, B, 1, 2, tid, nthr);   // d/dxi_y
    qsweep<N, false>(c.S, X2, 1, 2, tid, nthr);  // d/dxi_x
    __syncthreads();
    for (int e = tid; e < N3; e += nthr) {
      V[a * N3 + e] = X1[e];
      s[e] = fma(c.G[(0 + a) * N3 + e], X2[e], fma(c.G[(3 + a) * N3 + e], B[e], fma(c.G[(6 + a) * N3 + e], A[e], s[e])));
    }
    __syncthreads();
  }
  for (int e = tid; e < N3; e += nthr) s[e] = tau * s[e] / c.wd[e];
  __syncthreads();
  for (int a = 0; a < 3; ++a) {
    for (int e = tid; e < N3; e += nthr) {
      X1[e] = c.wd[e] * V[a * N3 + e];
      X2[e] = c.G[(0 + a) * N3 + e] * s[e];
      A[e] = c.G[(3 + a) * N3 + e] * s[e];
      B[e] = c.G[(6 + a) * N3 + e] * s[e];
    }
    __syncthreads();
    qsweep<N, true>(c.S, X1, 1, 2, tid, nthr);
    qsweep<N, true>(c.D, B, 1, 2, tid, nthr);
    qsweep<N, true>(c.S, A, 1, 2, tid, nthr);
    qsweep<N, true>(c.S, X2, 1, 2, tid, nthr);
    __syncthreads();
    for (int e = tid; e < N3; e += nthr) X1[e] += B[e];
    __syncthreads();
    qsweep<N, true>(c.S, X1, 1, 1, tid, nthr);
    qsweep<N, true>(c.D, A, 1, 1, tid, nthr);
    qsweep<N, true>(c.S, X2, 1, 1, tid, nthr);
    __syncthreads();
    for (int e = tid; e < N3; e += nthr) X1[e] += A[e];
    __syncthreads();
    qsweep<N, true>(c.S, X1, 1, 0, tid, nthr);
    qsweep<N, true>(c.D, X2, 1, 0, tid, nthr);
    __syncthreads();
    for (int e = tid; e < N3; e += nthr) out[a * N3 + e] = X1[e] + X2[e];
    __syncthreads();
  }
}

// z = M^{-1} r on one cell, three components, in place on z (which holds r on entry)
template <int N>
__device__ __forceinline__ void curv_minv(const CurvCell& c, double* z, int tid, int nthr) {
  constexpr int N3 = N * N * N;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    qsweep<N, true>(c.Si, z, 3, d, tid, nthr);
    __syncthreads();
  }
  for (int e = tid; e < 3 * N3; e += nthr) z[e] /= c.wd[e % N3];
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    qsweep<N, false>(c.Si, z, 3, d, tid, nthr);
    __syncthreads();
  }
}

template <int N>
__global__ void __launch_bounds__(64) k_curv_tau(const double* __restrict__ U, const ConvGeom g,
                                                 const double* __restrict__ wdet, double zeta, double dt,
                                                 double* __restrict__ tau, int64_t ncells) {
  constexpr int N3 = N * N * N;
  __shared__ double sU[3 * N3];
  const int tid = threadIdx.x;
  constexpr int nthr = 64;   // the launch size
  const int64_t cell = xcd_cell(blockIdx.x, gridDim.x);
  if (cell >= ncells) return;
  const int64_t Nd = ncells * N3;
  for (int e = tid; e < 3 * N3; e += nthr) sU[e] = U[(e / N3) * Nd + cell * N3 + e % N3];
  __syncthreads();
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    qsweep<N, false>(g.tab + g.S, sU, 3, d, tid, nthr);
    __syncthreads();
  }
  const double* wd = wdet + cell * 7 * N3 + 6 * N3;
  double v = 0.0, i0 = 0.0, i1 = 0.0, i2 = 0.0;
  for (int e = tid; e < N3; e += nthr) {
    v += wd[e];
    i0 = fma(wd[e], sU[e], i0);
    i1 = fma(wd[e], sU[N3 + e], i1);
    i2 = fma(wd[e], sU[2 * N3 + e], i2);
  }
  v = wave_total(v);
  i0 = wave_total(i0);
  i1 = wave_total(i1);
  i2 = wave_total(i2);
  if (tid == 0) tau[cell] = zeta * sqrt(i0 * i0 + i1 * i1 + i2 * i2) / v * cbrt(v) * dt;
}

template <int N>
__global__ void __launch_bounds__(64) k_curv_proj(const ConvGeom g, const double* __restrict__ wdet,
                                                  const double* __restrict__ taus, const double* __restrict__ rhs,
                                                  double* __restrict__ x, double rtol, int max_iter,
                                                  int* __restrict__ iters, int64_t ncells) {
  constexpr int N3 = N * N * N;
  __shared__ double sX[3 * N3], sR[3 * N3], sP[3 * N3], sQ[3 * N3], sW[8 * N3];
  const int tid = threadIdx.x;
  constexpr int nthr = 64;   // the launch size
  const int64_t cell = xcd_cell(blockIdx.x, gridDim.x);
  if (cell >= ncells) return;
  const int64_t Nd = ncells * N3;
  const CurvCell c{(ctab_ptr)(g.tab + g.S), (ctab_ptr)(g.tab + g.D), (ctab_ptr)(g.tab + g.Mi),
                   (gmem_ptr)(g.cmet + cell * 9 * N3), (gmem_ptr)(wdet + cell * 7 * N3 + 6 * N3)};
  const double tau = taus[cell];
  double bb = 0.0;
  for (int e = tid; e < 3 * N3; e += nthr) {
    const int64_t gi = (e / N3) * Nd + cell * N3 + e % N3;
    sX[e] = x[gi];
    sR[e] = rhs[gi];
    bb = fma(sR[e], sR[e], bb);
  }
  bb = wave_total(bb);
  __syncthreads();
  curv_mdd<N>(c, tau, sX, sQ, sW, tid, nthr);
  double rr = 0.0;
  for (int e = tid; e < 3 * N3; e += nthr) {
    sR[e] -= sQ[e];
    rr = fma(sR[e], sR[e], rr);
  }
  rr = wave_total(rr);
  const double tol2 = rtol * rtol * bb;
  int it = 0;
  if (rr > tol2) {
    __syncthreads();
    for (int e = tid; e < 3 * N3; e += nthr) sQ[e] = sR[e];
    __syncthreads();
    curv_minv<N>(c, sQ, tid, nthr);
    double rz = 0.0;
    for (int e = tid; e < 3 * N3; e += nthr) {
      sP[e] = sQ[e];
      rz = fma(sR[e], sQ[e], rz);
    }
    rz = wave_total(rz);
    __syncthreads();
    while (it < max_iter) {
      curv_mdd<N>(c, tau, sP, sQ, sW, tid, nthr);
      double pq = 0.0;
      for (int e = tid; e < 3 * N3; e += nthr) pq = fma(sP[e], sQ[e], pq);
      const double alpha = rz / wave_total(pq);
      rr = 0.0;
      for (int e = tid; e < 3 * N3; e += nthr) {
        sX[e] = fma(alpha, sP[e], sX[e]);
        sR[e] = fma(-alpha, sQ[e], sR[e]);
        rr = fma(sR[e], sR[e], rr);
      }
      rr = wave_total(rr);
      ++it;
      if (rr <= tol2) break;
      __syncthreads();
      for (int e = tid; e < 3 * N3; e += nthr) sQ[e] = sR[e];
      __syncthreads();
      curv_minv<N>(c, sQ, tid, nthr);
      double rz1 = 0.0;
      for (int e = tid; e < 3 * N3; e += nthr) rz1 = fma(sR[e], sQ[e], rz1);
      rz1 = wave_total(rz1);
      const double beta = rz1 / rz;
      rz = rz1;
      for (int e = tid; e < 3 * N3; e += nthr) sP[e] = fma(beta, sP[e], sQ[e]);
      __syncthreads();
    }
  }
  __syncthreads();
  for (int e = tid; e < 3 * N3; e += nthr) x[(e / N3) * Nd + cell * N3 + e % N3] = sX[e];
  if (iters && tid == 0) iters[cell] = it;
}

// ------------------------------------------------------ curved-cell metric
// Per cell quadrature point, w_q |det J| J^{-1} = w_q sgn(det J) adj(J) (nine
// values); per face point, the weighted normal w_q1 w_q2 |det J| J^{-T} e_d
// (Nanson's formula, along +xi_d), i.e. sgn(det J) times row d of adj(J),
// which only needs the two tangential columns of J.  Rows of a point: S/D at
// Gauss points, E (l(0), l(1)) and Gd (l'(0), l'(1)) at the ends.
struct FillTabs {
  const double *S, *D, *w, *E, *Gd;
};

template <int N, int Q>
__global__ void __launch_bounds__(256) k_conv_fill_cells(CurvMap m, int nx, int ny, int64_t ncells, FillTabs t,
                                                         double* __restrict__ cmet) {
  constexpr int Q3 = Q * Q * Q;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= ncells * Q3) return;
  const int64_t cell = gid / Q3;
  const int q = static_cast<int>(gid - cell * Q3);
  const int c[3] = {static_cast<int>(cell % nx), static_cast<int>((cell / nx) % ny),
                    static_cast<int>(cell / (static_cast<int64_t>(nx) * ny))};
  const int qi[3] = {q % Q, (q / Q) % Q, q / (Q * Q)};
  const double* val[3];
  const double* der[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    val[e] = t.S + qi[e] * N;
    der[e] = t.D + qi[e] * N;
  }
  double J[9];
  curv_jac_at<N>(m, c, val, der, J);
  double A[3][3];
#pragma unroll
  for (int e = 0; e < 3; ++e) adj_row(J, e, A[e]);
  const double det = J[0] * A[0][0] + J[3] * A[0][1] + J[6] * A[0][2];
  const double wq = (det < 0.0 ? -1.0 : 1.0) * t.w[qi[0]] * t.w[qi[1]] * t.w[qi[2]];
  double* out = cmet + cell * 9 * Q3 + q;
#pragma unroll
  for (int e = 0; e < 3; ++e)
#pragma unroll
    for (int b = 0; b < 3; ++b) out[(3 * e + b) * Q3] = wq * A[e][b];
}

template <int N, int Q>
__global__ void __launch_bounds__(256) k_conv_fill_faces(CurvMap m, int nx, int ny, int64_t ncells, FillTabs t,
                                                         double* __restrict__ fmet) {
  constexpr int Q2 = Q * Q;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= ncells * 6 * Q2) return;
  const int64_t cell = gid / (6 * Q2);
  const int r = static_cast<int>(gid - cell * 6 * Q2);
  const int f = r / Q2, pq = r % Q2;
  const int d = f >> 1, s = f & 1;
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  const int c[3] = {static_cast<int>(cell % nx), static_cast<int>((cell / nx) % ny),
                    static_cast<int>(cell / (static_cast<int64_t>(nx) * ny))};
  const double* val[3];
  const double* der[3];
  val[d] = t.E + s * N;
  der[d] = t.Gd + s * N;
  val[t1] = t.S + (pq % Q) * N;
  der[t1] = t.D + (pq % Q) * N;
  val[t2] = t.S + (pq / Q) * N;
  der[t2] = t.D + (pq / Q) * N;
  double J[9], nr[3];
  curv_jac_at<N>(m, c, val, der, J);
  adj_row(J, d, nr);
  const double det = J[d] * nr[0] + J[3 + d] * nr[1] + J[6 + d] * nr[2];
  const double wt = (det < 0.0 ? -1.0 : 1.0) * t.w[pq % Q] * t.w[pq / Q];
  double* out = fmet + (cell * 18 + f * 3) * Q2 + pq;
#pragma unroll
  for (int b = 0; b < 3; ++b) out[b * Q2] = wt * nr[b];
}

template <int N, int Q>
dgmf_status launch_fill_nq(const CurvMap& m, int nx, int ny, int64_t ncells, const FillTabs& t, double* cmet,
                           double* fmet, hipStream_t s) {
  const int64_t nc = ncells * Q * Q * Q, nf = ncells * 6 * Q * Q;
  if ((nc + 255) / 256 > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "mesh too large for one launch");
  hipLaunchKernelGGL((k_conv_fill_cells<N, Q>), dim3(static_cast<unsigned>((nc + 255) / 256)), dim3(256), 0, s, m,
                     nx, ny, ncells, t, cmet);
  DGMF_LAUNCH_CHECK("k_conv_fill_cells");
  hipLaunchKernelGGL((k_conv_fill_faces<N, Q>), dim3(static_cast<unsigned>((nf + 255) / 256)), dim3(256), 0, s, m,
                     nx, ny, ncells, t, fmet);
  DGMF_LAUNCH_CHECK("k_conv_fill_faces");
  return DGMF_OK;
}

template <int N, int Q>
dgmf_status launch_fwd_nq(const ConvGeom& g, const double* U, double* C, int64_t ncells, bool step, double dt,
                          hipStream_t s) {
  if (ncells > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "mesh too large for one launch");
  const bool curv = g.cmet != nullptr;
  if (curv && step) return fail(DGMF_UNSUPPORTED, "convective substep: curved cells are not supported");
  if (step)
    hipLaunchKernelGGL((k_conv_fwd<N, Q, true, false>), dim3(static_cast<unsigned>(ncells)),
                       dim3(CShape<N, Q>::THREADS), 0, s, U, C, g, ncells, dt);
  else if (curv)
    hipLaunchKernelGGL((k_conv_fwd<N, Q, false, true>), dim3(static_cast<unsigned>(ncells)),
                       dim3(CShape<N, Q>::THREADS), 0, s, U, C, g, ncells, dt);
  else
    hipLaunchKernelGGL((k_conv_fwd<N, Q, false, false>), dim3(static_cast<unsigned>(ncells)),
                       dim3(CShape<N, Q>::THREADS), 0, s, U, C, g, ncells, dt);
  DGMF_LAUNCH_CHECK("k_conv_fwd");
  return DGMF_OK;
}

template <int N, int Q>
dgmf_status launch_vjp_nq(const ConvGeom& g, const double* U, const double* W, double* G, int64_t ncells,
                          hipStream_t s) {
  if (ncells > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "mesh too large for one launch");
  if (g.cmet != nullptr)
    hipLaunchKernelGGL((k_conv_vjp<N, Q, true>), dim3(static_cast<unsigned>(ncells)), dim3(CShape<N, Q>::THREADS), 0,
                       s, U, W, G, g, ncells);
  else
    hipLaunchKernelGGL((k_conv_vjp<N, Q, false>), dim3(static_cast<unsigned>(ncells)), dim3(CShape<N, Q>::THREADS), 0,
                       s, U, W, G, g, ncells);
  DGMF_LAUNCH_CHECK("k_conv_vjp");
  return DGMF_OK;
}

template <int N>
dgmf_status launch_curv_v3_n(bool grad, const ConvGeom& g, const double* in, double* out, int64_t ncells,
                             hipStream_t s) {
  if (ncells > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "mesh too large for one launch");
  if (grad) {
    hipLaunchKernelGGL((k_curv_grad<N, N>), dim3(static_cast<unsigned>(ncells)), dim3(CShape<N, N>::THREADS), 0, s,
                       in, out, g, ncells);
    DGMF_LAUNCH_CHECK("k_curv_grad");
  } else {
    hipLaunchKernelGGL((k_curv_div<N, N>), dim3(static_cast<unsigned>(ncells)), dim3(CShape<N, N>::THREADS), 0, s,
                       in, out, g, ncells);
    DGMF_LAUNCH_CHECK("k_curv_div");
  }
  return DGMF_OK;
}

template <int N>
dgmf_status launch_curv_cell_n(bool proj, const ConvGeom& g, const double* wdet, const double* u, double zeta,
                               double dt, double* tau, const double* taus, const double* rhs, double* x, double rtol,
                               int max_iter, int* iters, int64_t ncells, hipStream_t s) {
  if (ncells > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "mesh too large for one launch");
  if (proj) {
    hipLaunchKernelGGL((k_curv_proj<N>), dim3(static_cast<unsigned>(ncells)), dim3(64), 0, s, g, wdet, taus, rhs, x,
                       rtol, max_iter, iters, ncells);
    DGMF_LAUNCH_CHECK("k_curv_proj");
  } else {
    hipLaunchKernelGGL((k_curv_tau<N>), dim3(static_cast<unsigned>(ncells)), dim3(64), 0, s, u, g, wdet, zeta, dt,
                       tau, ncells);
    DGMF_LAUNCH_CHECK("k_curv_tau");
  }
  return DGMF_OK;
}

// ------------------------------------- viscous coupling on curved cells
// The component coupling nu C(u) of the viscous operator in the
// symmetric-gradient form (Sec. 3.2, implicit viscous step, s = 1,
// F^nu(u) = 2 nu eps(u)) on iso-parametric curved cells; the rest of that
// operator is the scalar SIPG Helmholtz operator of every component (the
// stored-metric apply).  With d_b u_a the physical gradient, k+1 Gauss points
// per direction, w|J| the weighted Jacobian determinant at a cell point, nw
// the weighted outward normal (w dA n) at a face point and [u] the own trace
// minus the neighbour's:
//   (C u)_{c,i} = sum_q w|J| sum_a d_a phi_i d_c u_a
//     - sum_p [ 1/2 nw_c (grad phi_i . [u]) + 1/2 phi_i (nw . d_c u_own + nw . d_c u_nb) ]   interior faces
//     - sum_p [ nw_c (grad phi_i . u) + phi_i (nw . d_c u) ]                                  Dirichlet faces
// (nw . d_c u = sum_a nw_a d_c u_a); homogeneous Neumann sides add nothing.
// The Jacobian is evaluated in closed form at every point (curv_map.h), so
// nothing is stored per point.  Reference gradients at face points: the
// tangential ones from the nodal trace plane, the normal one from the nodal
// normal-derivative plane (l'(0) or l'(1) along every normal line), for the
// own cell and, from global memory, its neighbour.  One cell per workgroup.
struct EpsCurvGeom {
  ConvGeom g;    // tab: S, D, w at the Gauss points; E (l(0), l(1)) and Gd (l'(0), l'(1)) at offsets E, Gd
  CurvMap m;
  int E, Gd;
};

// node (l, j, i) at position m along the normal line of face direction d through face-plane entry (p1, p2)
template <int N>
__device__ __forceinline__ int line_node(int d, int m, int p1, int p2) {
  if (d == 0) return (p2 * N + p1) * N + m;
  if (d == 1) return (p2 * N + m) * N + p1;
  return (m * N + p2) * N + p1;
}

// J of a point from the per-direction values sg[e] = sig_e and dsg[e] = sig_e'
// there (curv_map.h), with the cell sizes h[e]; returns J^{-1} and det J.
__device__ __forceinline__ double jinv_from(const CurvMap& m, const double h[3], const double sg[3],
                                            const double dsg[3], double Ji[3][3]) {
  double J[9];
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int d = 0; d < 3; ++d) J[r * 3 + d] = r == d ? h[r] : m.amp * m.len[r] * dsg[d] * sg[3 - r - d];
  double A[3][3];
#pragma unroll
  for (int e = 0; e < 3; ++e) adj_row(J, e, A[e]);
  const double det = J[0] * A[0][0] + J[3] * A[0][1] + J[6] * A[0][2];
  const double inv = 1.0 / det;
#pragma unroll
  for (int e = 0; e < 3; ++e)
#pragma unroll
    for (int b = 0; b < 3; ++b) Ji[e][b] = A[e][b] * inv;
  return det;
}

// Reference gradient of the nodal field sIn[N^3] at this thread's quadrature
// z-column (gx, gy, gz).  T1 (2 N^2 Q) and T2 (3 N Q^2) are LDS scratch; ends
// with a barrier.
template <int N, int Q>
__device__ __forceinline__ void grad3(const double* __restrict__ S, const double* __restrict__ D, const double* sIn,
                                      double* T1, double* T2, int tid, int nthr, bool own, int qx, int qy,
                                      double (&gx)[Q], double (&gy)[Q], double (&gz)[Q]) {
  constexpr int N2 = N * N, Q2 = Q * Q;
  for (int job = tid; job < N2; job += nthr) {          // x: line (l, j), values and x-derivatives
    double v[N];
#pragma unroll
    for (int i = 0; i < N; ++i) v[i] = sIn[job * N + i];
#pragma unroll kSweepUnroll<N, Q>
    for (int q = 0; q < Q; ++q) {
      double a = 0, b = 0;
#pragma unroll
      for (int i = 0; i < N; ++i) {
        a = fma(S[q * N + i], v[i], a);
        b = fma(D[q * N + i], v[i], b);
      }
      T1[job * Q + q] = a;
      T1[N2 * Q + job * Q + q] = b;
    }
  }
  __syncthreads();
  for (int job = tid; job < 2 * N * Q; job += nthr) {   // y: (input plane, l, qx)
    const int qxx = job % Q, l = (job / Q) % N, w = job / (N * Q);
    double v[N];
#pragma unroll
    for (int j = 0; j < N; ++j) v[j] = T1[w * N2 * Q + (l * N + j) * Q + qxx];
#pragma unroll kSweepUnroll<N, Q>
    for (int q = 0; q < Q; ++q) {
      double a = 0, b = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) {
        a = fma(S[q * N + j], v[j], a);
        b = fma(D[q * N + j], v[j], b);
      }
      if (w == 0) {
        T2[(l * Q + q) * Q + qxx] = a;                // S_y S_x u
        T2[N * Q2 + (l * Q + q) * Q + qxx] = b;       // D_y S_x u
      } else {
        T2[2 * N * Q2 + (l * Q + q) * Q + qxx] = a;   // S_y D_x u
      }
    }
  }
  __syncthreads();
  if (own) {
#pragma unroll
    for (int q = 0; q < Q; ++q) gx[q] = gy[q] = gz[q] = 0.0;
#pragma unroll kSweepUnroll<N, Q>
    for (int l = 0; l < N; ++l) {
      const double a = T2[(l * Q + qy) * Q + qx], b = T2[N * Q2 + (l * Q + qy) * Q + qx],
                   c = T2[2 * N * Q2 + (l * Q + qy) * Q + qx];
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        gz[q] = fma(D[q * N + l], a, gz[q]);
        gy[q] = fma(S[q * N + l], b, gy[q]);
        gx[q] = fma(S[q * N + l], c, gx[q]);
      }
    }
  }
  __syncthreads();
}

template <int N>
__global__ void __launch_bounds__((CShape<N, N>::THREADS)) k_eps_curved(const double* __restrict__ U,
                                                                      double* __restrict__ out,
                                                                      const EpsCurvGeom eg, double nu,
                                                                      int64_t ncells) {
  constexpr int Q = N;
  using SH = CShape<N, Q>;
  constexpr int N2 = SH::N2, N3 = SH::N3, Q2 = SH::Q2;
  constexpr int XC = 2 * N2 * Q + 3 * N * Q2 > 3 * N * Q2 + 2 * N2 * Q ? 2 * N2 * Q + 3 * N * Q2
                                                                         : 3 * N * Q2 + 2 * N2 * Q;
  // faces: nodal planes [side][comp][value | normal derivative], first sweep [side][comp][3],
  // face-point data [side][comp][4], fluxes [comp][4], lift stage [comp][4] and lifted planes [comp][2]
  constexpr int XF = 12 * N2 + 18 * N * Q + 24 * Q2 + 12 * Q2 + 12 * N * Q + 6 * N2;
  constexpr int X = XC > XF ? XC : XF;
  __shared__ double sU[3 * N3];
  __shared__ double sO[3 * N3];
  __shared__ double sX[X];
  __shared__ double sSG[3][Q + 2], sDSG[3][Q + 2];
  const ConvGeom& g = eg.g;
  const CurvMap& m = eg.m;
  const int tid = threadIdx.x;
  constexpr int nthr = SH::THREADS;
  const int64_t cell = xcd_cell(blockIdx.x, gridDim.x);
  if (cell >= ncells) return;
  const int64_t Nd = ncells * N3;
  // the 1D tables in LDS: read from there they leave the scalar registers to
  // the map and the geometry (read as scalar loads they spilled)
  __shared__ double sT[2 * N * Q + Q + 4 * N];
  for (int e = tid; e < N * Q; e += nthr) {
    sT[e] = g.tab[g.S + e];
    sT[N * Q + e] = g.tab[g.D + e];
  }
  for (int e = tid; e < Q; e += nthr) sT[2 * N * Q + e] = g.tab[g.w + e];
  for (int e = tid; e < 2 * N; e += nthr) {
    sT[2 * N * Q + Q + e] = g.tab[eg.E + e];
    sT[2 * N * Q + Q + 2 * N + e] = g.tab[eg.Gd + e];
  }
  const double* S = sT;
  const double* D = sT + N * Q;
  const double* W = sT + 2 * N * Q;
  const double* E = sT + 2 * N * Q + Q;
  const double* Gd = sT + 2 * N * Q + Q + 2 * N;
  CellGeo cg;
  conv_cell(g, cell, cg);
  for (int e = tid; e < 3 * N3; e += nthr) {
    const int a = e / N3, r = e % N3;
    sU[e] = U[a * Nd + cell * N3 + r];
  }
  // sig and sig' of the map per direction at the Gauss points (0..Q-1) and the ends (Q, Q+1)
  for (int e = tid; e < 3 * (Q + 2); e += nthr) {
    const int dir = e / (Q + 2), t = e % (Q + 2);
    const double* val = t < Q ? S + t * N : E + (t - Q) * N;
    const double* der = t < Q ? D + t * N : Gd + (t - Q) * N;
    curv_sig_at<N>(m, dir, cg.c[dir], val, der, sSG[dir][t], sDSG[dir][t]);
  }
  __syncthreads();
  const bool own = tid < Q2;
  const int qx = tid % Q, qy = (tid / Q) % Q;
  // ---- cell term: fe_c[r] = w|J| sum_a Ji[r][a] d_c u_a, lifted by the reference gradients
  double gr[3][3][Q];   // [component][reference direction][qz]; becomes fe[c][r][qz]
#pragma unroll
  for (int a = 0; a < 3; ++a)
    grad3<N, Q>(S, D, sU + a * N3, sX, sX + 2 * N2 * Q, tid, nthr, own, qx, qy, gr[a][0], gr[a][1], gr[a][2]);
  if (own) {
#pragma unroll
    for (int q = 0; q < Q; ++q) {
      const int qi[3] = {qx, qy, q};
      double sg[3], dsg[3], Ji[3][3];
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        sg[e] = sSG[e][qi[e]];
        dsg[e] = sDSG[e][qi[e]];
      }
      const double det = jinv_from(m, cg.h, sg, dsg, Ji);
      const double wj = fabs(det) * W[qx] * W[qy] * W[q];
      double Gp[3][3];   // Gp[a][b] = d_b u_a
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          Gp[a][b] = fma(gr[a][0][q], Ji[0][b], fma(gr[a][1][q], Ji[1][b], gr[a][2][q] * Ji[2][b]));
#pragma unroll
      for (int c = 0; c < 3; ++c)
#pragma unroll
        for (int r = 0; r < 3; ++r)
          gr[c][r][q] = wj * fma(Ji[r][0], Gp[0][c], fma(Ji[r][1], Gp[1][c], Ji[r][2] * Gp[2][c]));
    }
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
    cell_lift_grad<N, Q>(S, D, gr[c][0], gr[c][1], gr[c][2], own, qx, qy, sX, sX + 3 * N * Q2, sO + c * N3, nu, tid,
                         nthr);
  // ---- faces
  double* P = sX;                    // [side][comp][2][N2]
  double* F1 = P + 12 * N2;          // [side][comp][3][N][Q]
  double* F2 = F1 + 18 * N * Q;      // [side][comp][4][Q2]: value, d/dt2, d/dt1, d/dn
  double* R = F2 + 24 * Q2;          // [comp][4][Q2]: value flux, reference gradient flux along t1, t2, d
  double* L1 = R + 12 * Q2;          // [comp][4][N][Q]
  double* LP = L1 + 12 * N * Q;      // [comp][2][N2]: tangential lift, normal lift
#pragma unroll 1
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1, s = f & 1;
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const int64_t nb = conv_nb(g, cg, cell, d, s);
    if (nb < 0 && ((g.neu >> f) & 1)) continue;   // homogeneous Neumann side: no term
    const bool inner = nb >= 0;
    const int nsides = inner ? 2 : 1;
    const double* gs = Gd + s * N;          // l'(end) of the own side
    const double* gn = Gd + (1 - s) * N;    // of the neighbour side
    for (int e = tid; e < nsides * 3 * N2; e += nthr) {
      const int side = e / (3 * N2), a = (e / N2) % 3, p = e % N2, p1 = p % N, p2 = p / N;
      double v = 0.0, dn = 0.0;
      if (side == 0) {
        const double* u = sU + a * N3;
#pragma unroll
        for (int mm = 0; mm < N; ++mm) dn = fma(gs[mm], u[line_node<N>(d, mm, p1, p2)], dn);
        v = u[line_node<N>(d, s ? N - 1 : 0, p1, p2)];
      } else {
        const double* u = U + a * Nd + nb * N3;
#pragma unroll
        for (int mm = 0; mm < N; ++mm) dn = fma(gn[mm], u[line_node<N>(d, mm, p1, p2)], dn);
        v = u[line_node<N>(d, s ? 0 : N - 1, p1, p2)];
      }
      P[((side * 3 + a) * 2 + 0) * N2 + p] = v;
      P[((side * 3 + a) * 2 + 1) * N2 + p] = dn;
    }
    __syncthreads();
    for (int job = tid; job < nsides * 3 * N; job += nthr) {   // along t1: (side, comp, p2)
      const int p2 = job % N, sa = job / N;
      double v[N], w[N];
#pragma unroll
      for (int p = 0; p < N; ++p) {
        v[p] = P[(sa * 2 + 0) * N2 + p2 * N + p];
        w[p] = P[(sa * 2 + 1) * N2 + p2 * N + p];
      }
#pragma unroll kSweepUnroll<N, Q>
      for (int q = 0; q < Q; ++q) {
        double a0 = 0, a1 = 0, a2 = 0;
#pragma unroll
        for (int p = 0; p < N; ++p) {
          a0 = fma(S[q * N + p], v[p], a0);
          a1 = fma(D[q * N + p], v[p], a1);
          a2 = fma(S[q * N + p], w[p], a2);
        }
        F1[((sa * 3 + 0) * N + p2) * Q + q] = a0;
        F1[((sa * 3 + 1) * N + p2) * Q + q] = a1;
        F1[((sa * 3 + 2) * N + p2) * Q + q] = a2;
      }
    }
    __syncthreads();
    for (int job = tid; job < nsides * 3 * Q; job += nthr) {   // along t2: (side, comp, q1)
      const int q1 = job % Q, sa = job / Q;
      double v0[N], v1[N], v2[N];
#pragma unroll
      for (int p = 0; p < N; ++p) {
        v0[p] = F1[((sa * 3 + 0) * N + p) * Q + q1];
        v1[p] = F1[((sa * 3 + 1) * N + p) * Q + q1];
        v2[p] = F1[((sa * 3 + 2) * N + p) * Q + q1];
      }
#pragma unroll kSweepUnroll<N, Q>
      for (int q = 0; q < Q; ++q) {
        double val = 0, dt2 = 0, dt1 = 0, dnn = 0;
#pragma unroll
        for (int p = 0; p < N; ++p) {
          val = fma(S[q * N + p], v0[p], val);
          dt2 = fma(D[q * N + p], v0[p], dt2);
          dt1 = fma(S[q * N + p], v1[p], dt1);
          dnn = fma(S[q * N + p], v2[p], dnn);
        }
        F2[((sa * 4 + 0) * Q + q) * Q + q1] = val;
        F2[((sa * 4 + 1) * Q + q) * Q + q1] = dt2;
        F2[((sa * 4 + 2) * Q + q) * Q + q1] = dt1;
        F2[((sa * 4 + 3) * Q + q) * Q + q1] = dnn;
      }
    }
    __syncthreads();
    // fluxes at the face points
    double sgn_nb = 0.0, dsg_nb = 0.0, h_nb = 0.0;
    if (inner) {
      const int nd = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
      int cc = cg.c[d] + (s ? 1 : -1);
      cc = cc < 0 ? nd - 1 : (cc >= nd ? 0 : cc);
      curv_sig_at<N>(m, d, cc, E + (1 - s) * N, Gd + (1 - s) * N, sgn_nb, dsg_nb);
      h_nb = m.h[d][cc];
    }
    for (int pq = tid; pq < Q2; pq += nthr) {
      const int q1 = pq % Q, q2 = pq / Q;
      double sg[3], dsg[3], Jo[3][3], Je[3][3];
      sg[d] = sSG[d][Q + s];
      dsg[d] = sDSG[d][Q + s];
      sg[t1] = sSG[t1][q1];
      dsg[t1] = sDSG[t1][q1];
      sg[t2] = sSG[t2][q2];
      dsg[t2] = sDSG[t2][q2];
      const double det = jinv_from(m, cg.h, sg, dsg, Jo);
      // weighted outward normal: w_t1 w_t2 det J J^{-T} e_d, oriented out of this cell
      const double wn = (s ? 1.0 : -1.0) * W[q1] * W[q2] * fabs(det);
      const double nw[3] = {wn * Jo[d][0], wn * Jo[d][1], wn * Jo[d][2]};
      double uo[3], Go[3][3];
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const double* Fa = F2 + (0 * 3 + a) * 4 * Q2 + pq;
        double gref[3];
        uo[a] = Fa[0];
        gref[t2] = Fa[Q2];
        gref[t1] = Fa[2 * Q2];
        gref[d] = Fa[3 * Q2];
#pragma unroll
        for (int b = 0; b < 3; ++b) Go[a][b] = fma(gref[0], Jo[0][b], fma(gref[1], Jo[1][b], gref[2] * Jo[2][b]));
      }
      double jmp[3], fac;
      double Rv[3];   // value flux per output component, before the factor -fac nu
      if (inner) {
        double h3[3] = {cg.h[0], cg.h[1], cg.h[2]};
        h3[d] = h_nb;
        sg[d] = sgn_nb;
        dsg[d] = dsg_nb;
        jinv_from(m, h3, sg, dsg, Je);
        double ue[3], Ge[3][3];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const double* Fa = F2 + (1 * 3 + a) * 4 * Q2 + pq;
          double gref[3];
          ue[a] = Fa[0];
          gref[t2] = Fa[Q2];
          gref[t1] = Fa[2 * Q2];
          gref[d] = Fa[3 * Q2];
#pragma unroll
          for (int b = 0; b < 3; ++b) Ge[a][b] = fma(gref[0], Je[0][b], fma(gref[1], Je[1][b], gref[2] * Je[2][b]));
          jmp[a] = uo[a] - ue[a];
        }
#pragma unroll
        for (int c = 0; c < 3; ++c)
          Rv[c] = fma(nw[0], Go[0][c] + Ge[0][c], fma(nw[1], Go[1][c] + Ge[1][c], nw[2] * (Go[2][c] + Ge[2][c])));
        fac = 0.5;
      } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) jmp[a] = uo[a];
#pragma unroll
        for (int c = 0; c < 3; ++c) Rv[c] = fma(nw[0], Go[0][c], fma(nw[1], Go[1][c], nw[2] * Go[2][c]));
        fac = 1.0;
      }
      double z[3];   // sum_b Ji[r][b] [u]_b: grad phi . [u] = sum_r dphi/dxi_r z_r
#pragma unroll
      for (int r = 0; r < 3; ++r) z[r] = fma(Jo[r][0], jmp[0], fma(Jo[r][1], jmp[1], Jo[r][2] * jmp[2]));
      const double sc = -fac * nu;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        double* Rc = R + c * 4 * Q2 + pq;
        Rc[0] = sc * Rv[c];
        Rc[Q2] = sc * nw[c] * z[t1];
        Rc[2 * Q2] = sc * nw[c] * z[t2];
        Rc[3 * Q2] = sc * nw[c] * z[d];
      }
    }
    __syncthreads();
    for (int job = tid; job < 3 * Q; job += nthr) {   // transposed, along t2: [q2][q1] -> [p2][q1]
      const int q1 = job % Q, c = job / Q;
      double v[4][Q];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < Q; ++q) v[k][q] = R[(c * 4 + k) * Q2 + q * Q + q1];
#pragma unroll kSweepUnroll<N, Q>
      for (int p = 0; p < N; ++p) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          a0 = fma(S[q * N + p], v[0][q], a0);
          a1 = fma(S[q * N + p], v[1][q], a1);
          a2 = fma(D[q * N + p], v[2][q], a2);
          a3 = fma(S[q * N + p], v[3][q], a3);
        }
        L1[((c * 4 + 0) * N + p) * Q + q1] = a0;
        L1[((c * 4 + 1) * N + p) * Q + q1] = a1;
        L1[((c * 4 + 2) * N + p) * Q + q1] = a2;
        L1[((c * 4 + 3) * N + p) * Q + q1] = a3;
      }
    }
    __syncthreads();
    for (int job = tid; job < 3 * N; job += nthr) {   // transposed, along t1: [p2][q1] -> [p2][p1]
      const int p2 = job % N, c = job / N;
      double v[4][Q];
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int q = 0; q < Q; ++q) v[k][q] = L1[((c * 4 + k) * N + p2) * Q + q];
#pragma unroll kSweepUnroll<N, Q>
      for (int p1 = 0; p1 < N; ++p1) {
        double tg = 0, nn = 0;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
          tg = fma(S[q * N + p1], v[0][q] + v[2][q], fma(D[q * N + p1], v[1][q], tg));
          nn = fma(S[q * N + p1], v[3][q], nn);
        }
        LP[(c * 2 + 0) * N2 + p2 * N + p1] = tg;
        LP[(c * 2 + 1) * N2 + p2 * N + p1] = nn;
      }
    }
    __syncthreads();
    for (int job = tid; job < 3 * N2; job += nthr) {  // onto the face nodes and along the normal lines
      const int c = job / N2, p = job % N2, p1 = p % N, p2 = p / N;
      const double tg = LP[(c * 2 + 0) * N2 + p], nn = LP[(c * 2 + 1) * N2 + p];
      double* o = sO + c * N3;
#pragma unroll
      for (int mm = 0; mm < N; ++mm) o[line_node<N>(d, mm, p1, p2)] = fma(gs[mm], nn, o[line_node<N>(d, mm, p1, p2)]);
      o[line_node<N>(d, s ? N - 1 : 0, p1, p2)] += tg;
    }
    __syncthreads();
  }
  for (int e = tid; e < 3 * N3; e += nthr) {
    const int a = e / N3, r = e % N3;
    out[a * Nd + cell * N3 + r] += sO[e];
  }
}

template <int N>
dgmf_status launch_eps_curved_n(const EpsCurvGeom& eg, const double* u, double* out, double nu, int64_t ncells,
                                hipStream_t s) {
  if (ncells > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "mesh too large for one launch");
  hipLaunchKernelGGL((k_eps_curved<N>), dim3(static_cast<unsigned>(ncells)), dim3(CShape<N, N>::THREADS), 0, s, u,
                     out, eg, nu, ncells);
  DGMF_LAUNCH_CHECK("k_eps_curved");
  return DGMF_OK;
}

}  // namespace

// Supported (n, n_q): the paper's floor(3k/2)+1 and floor(3(k+1)/2) for k = 1..6
// (k = 7 would need more than 64 KiB of LDS per workgroup in this layout).
#define DGMF_CONV_CASES(X) \
  X(2, 2) X(2, 3) X(3, 4) X(4, 5) X(4, 6) X(5, 7) X(6, 8) X(6, 9) X(7, 10) X(7, 11)
// the curved V3c operators: n_q = n = k+1 for k = 2..7 (k = 1 is (2, 2) above)
#define DGMF_QN_CASES(X) X(3, 3) X(4, 4) X(5, 5) X(6, 6) X(7, 7) X(8, 8)

bool conv_supported(int n, int nq) {
#define X(a, b) if (n == a && nq == b) return true;
  DGMF_CONV_CASES(X)
#undef X
  return false;
}

dgmf_status launch_conv_fwd(int n, int nq, const ConvGeom& g, const double* U, double* C, int64_t ncells,
                            bool step, double dt, hipStream_t s) {
#define X(a, b) if (n == a && nq == b) return launch_fwd_nq<a, b>(g, U, C, ncells, step, dt, s);
  DGMF_CONV_CASES(X)
#undef X
  return fail(DGMF_UNSUPPORTED, "convective: (n, n_q) = (%d, %d) not built", n, nq);
}

dgmf_status launch_conv_vjp(int n, int nq, const ConvGeom& g, const double* U, const double* W, double* G,
                            int64_t ncells, hipStream_t s) {
#define X(a, b) if (n == a && nq == b) return launch_vjp_nq<a, b>(g, U, W, G, ncells, s);
  DGMF_CONV_CASES(X)
#undef X
  return fail(DGMF_UNSUPPORTED, "convective: (n, n_q) = (%d, %d) not built", n, nq);
}

dgmf_status launch_conv_fill_curved(int n, int nq, const double* const x0[3], const double* const h[3],
                                    const double lo[3], const double len[3], double amp, int nx, int ny,
                                    int64_t ncells, const double* tab, const int off[6], double* cmet, double* fmet,
                                    hipStream_t s) {
  CurvMap m{};
  for (int d = 0; d < 3; ++d) {
    m.x0[d] = x0[d];
    m.h[d] = h[d];
    m.lo[d] = lo[d];
    m.len[d] = len[d];
  }
  m.amp = amp;
  m.nodes = tab + off[0];
  const FillTabs t{tab + off[1], tab + off[2], tab + off[3], tab + off[4], tab + off[5]};
#define X(a, b) if (n == a && nq == b) return launch_fill_nq<a, b>(m, nx, ny, ncells, t, cmet, fmet, s);
  DGMF_CONV_CASES(X)
  DGMF_QN_CASES(X)
#undef X
  return fail(DGMF_UNSUPPORTED, "convective: (n, n_q) = (%d, %d) not built", n, nq);
}

dgmf_status launch_curv_v3(int n, bool grad, const ConvGeom& g, const double* in, double* out, int64_t ncells,
                           hipStream_t s) {
  switch (n) {
    case 2: return launch_curv_v3_n<2>(grad, g, in, out, ncells, s);
    case 3: return launch_curv_v3_n<3>(grad, g, in, out, ncells, s);
    case 4: return launch_curv_v3_n<4>(grad, g, in, out, ncells, s);
    case 5: return launch_curv_v3_n<5>(grad, g, in, out, ncells, s);
    case 6: return launch_curv_v3_n<6>(grad, g, in, out, ncells, s);
    case 7: return launch_curv_v3_n<7>(grad, g, in, out, ncells, s);
    case 8: return launch_curv_v3_n<8>(grad, g, in, out, ncells, s);
    default: return fail(DGMF_UNSUPPORTED, "curved V3c operators: n = %d not built", n);
  }
}

dgmf_status launch_curv_cell(int n, bool proj, const ConvGeom& g, const double* wdet, const double* u, double zeta,
                             double dt, double* tau, const double* taus, const double* rhs, double* x, double rtol,
                             int max_iter, int* iters, int64_t ncells, hipStream_t s) {
#define X(a)                                                                                                    \
  if (n == a)                                                                                                   \
    return launch_curv_cell_n<a>(proj, g, wdet, u, zeta, dt, tau, taus, rhs, x, rtol, max_iter, iters, ncells, s);
  X(2) X(3) X(4) X(5) X(6) X(7)
#undef X
  return fail(DGMF_UNSUPPORTED, "curved div-div penalty / projection: n = %d not built", n);
}

dgmf_status launch_eps_curved(int n, const ConvGeom& g, const double* const x0[3], const double* const h[3],
                              const double lo[3], const double len[3], double amp, int off_nodes, int off_e,
                              int off_gd, const double* u, double* out, double nu, int64_t ncells, hipStream_t s) {
  EpsCurvGeom eg{};
  eg.g = g;
  for (int d = 0; d < 3; ++d) {
    eg.m.x0[d] = x0[d];
    eg.m.h[d] = h[d];
    eg.m.lo[d] = lo[d];
    eg.m.len[d] = len[d];
  }
  eg.m.amp = amp;
  eg.m.nodes = g.tab + off_nodes;
  eg.E = off_e;
  eg.Gd = off_gd;
  switch (n) {
    case 2: return launch_eps_curved_n<2>(eg, u, out, nu, ncells, s);
    case 3: return launch_eps_curved_n<3>(eg, u, out, nu, ncells, s);
    case 4: return launch_eps_curved_n<4>(eg, u, out, nu, ncells, s);
    case 5: return launch_eps_curved_n<5>(eg, u, out, nu, ncells, s);
    case 6: return launch_eps_curved_n<6>(eg, u, out, nu, ncells, s);
    case 7: return launch_eps_curved_n<7>(eg, u, out, nu, ncells, s);
    default: return fail(DGMF_UNSUPPORTED, "curved viscous operator: n = %d not built", n);
  }
}

}  // namespace dgmf
