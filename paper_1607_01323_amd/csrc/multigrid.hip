// Level transfers and vector kernels of the geometric multigrid V-cycle
// (Sec. 5.1, Poisson solver) on box-mesh hierarchies (gfx950).
//
// Transfers are the tensorial embedding of a mother cell's nodal polynomial
// into its children: along a halved direction d, child s of the mother takes
// the values E_d[s][i][a] = l_a((s + xi_i)/2) times the mother's nodal values
// (a direction that is not halved uses the identity).  Prolongation adds
//   x_child += (E_z[sz] (x) E_y[sy] (x) E_x[sx]) x_mother
// to the fine vector; restriction is its transpose applied to the fine
// residual b - A x,
//   b_mother = sum over children (E_z[sz] (x) E_y[sy] (x) E_x[sx])^T (b - t)_child.
// Both run one mother cell per wavefront with the children staged in the
// wavefront's LDS slice and three 1D sweeps (x, y, z), so each fine value is
// read or written once; a mother owns its children, so no atomics.
//
// The smoother and the coarse solver are Chebyshev accelerations of point
// Jacobi (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1) in
// three-term form on the iterate: x_1 = x_0 + dinv (b - A x_0) / theta and
//   x_{k+1} = x_k + c1_k (x_k - x_{k-1}) + c2_k dinv (b - A x_k);
// the update is fused into the apply kernel's store (axis-aligned and
// stored-metric levels alike); k_mg_cheb_vec applies it after a plain apply
// for an operator without that fusion.
#include "internal.h"

namespace dgmf {
namespace {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

#define MG_GRID_STRIDE(i, N) \
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < (N); i += static_cast<int64_t>(gridDim.x) * blockDim.x)

constexpr int kMgVecBlocks = 2048;

template <int N, typename T>
struct XShape {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int SLICE = 14 * N3;   // children (8 N^3) + after one sweep (4 N^3) + after two (2 N^3)
  static constexpr int BYTES = SLICE * static_cast<int>(sizeof(T));
  static constexpr int WAVES = BYTES * 4 <= 60000 ? 4 : (BYTES * 2 <= 60000 ? 2 : 1);
};

struct XferCells {
  int cnx, cny, cnz;      // coarse cell counts
  int fnx, fny;           // fine cell counts in x, y
  int r[3];               // 1 or 2 per direction
};

__device__ __forceinline__ int64_t child_cell(const XferCells& g, int CX, int CY, int CZ, int sx, int sy, int sz) {
  return (static_cast<int64_t>(CZ * g.r[2] + sz) * g.fny + (CY * g.r[1] + sy)) * g.fnx + (CX * g.r[0] + sx);
}

// xf += P xc, one mother cell per wavefront.
template <int N, typename T>
__global__ void __launch_bounds__(256) k_mg_prolong(const T* __restrict__ xc, T* __restrict__ xf,
                                                    const T* __restrict__ etab, const XferCells g, int64_t ncoarse,
                                                    const int* stop) {
  using SH = XShape<N, T>;
  constexpr int N2 = SH::N2, N3 = SH::N3;
  __shared__ T s_tab[6 * N2];
  __shared__ T s_all[SH::WAVES * SH::SLICE];
  if (stop && *stop) return;
  for (int e = threadIdx.x; e < 6 * N2; e += blockDim.x) s_tab[e] = etab[e];
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t C = static_cast<int64_t>(blockIdx.x) * SH::WAVES + wave;
  if (C >= ncoarse) return;
  T* in = s_all + wave * SH::SLICE;     // N3
  T* A = in + N3;                         // rx N3
  T* B = A + 2 * N3;                      // rx ry N3
  const int CX = static_cast<int>(C % g.cnx);
  const int CY = static_cast<int>((C / g.cnx) % g.cny);
  const int CZ = static_cast<int>(C / (static_cast<int64_t>(g.cnx) * g.cny));
  const int rx = g.r[0], ry = g.r[1], rz = g.r[2];
  for (int e = lane; e < N3; e += 64) in[e] = xc[C * N3 + e];
  wave_sync();
  for (int e = lane; e < rx * N3; e += 64) {           // A[sx][l][j][i] = sum_a Ex[sx][i][a] in[l][j][a]
    const int i = e % N, lj = (e / N) % N2, sx = e / N3;
    const T* ex = s_tab + (0 * 2 + sx) * N2 + i * N;
    const T* src = in + lj * N;
    T acc = 0;
#pragma unroll
    for (int a = 0; a < N; ++a) acc = fma(ex[a], src[a], acc);
    A[e] = acc;
  }
  wave_sync();
  for (int e = lane; e < ry * rx * N3; e += 64) {      // B[sy][sx][l][j][i] = sum_b Ey[sy][j][b] A[sx][l][b][i]
    const int i = e % N, j = (e / N) % N, l = (e / N2) % N, sx = (e / N3) % rx, sy = e / (rx * N3);
    const T* ey = s_tab + (1 * 2 + sy) * N2 + j * N;
    const T* src = A + sx * N3 + l * N2 + i;
    T acc = 0;
#pragma unroll
    for (int b = 0; b < N; ++b) acc = fma(ey[b], src[b * N], acc);
    B[e] = acc;
  }
  wave_sync();
  const int nch = rx * ry * rz;
  for (int e = lane; e < nch * N3; e += 64) {          // child-major, node index fastest: coalesced
    const int r = e % N3, ch = e / N3;
    const int sx = ch % rx, sy = (ch / rx) % ry, sz = ch / (rx * ry);
    const int l = r / N2, ji = r % N2;
    const T* ez = s_tab + (2 * 2 + sz) * N2 + l * N;
    const T* src = B + (sy * rx + sx) * N3 + ji;
    T acc = 0;
#pragma unroll
    for (int c = 0; c < N; ++c) acc = fma(ez[c], src[c * N2], acc);
    T* dst = xf + child_cell(g, CX, CY, CZ, sx, sy, sz) * N3 + r;
    *dst += acc;
  }
}

// bc = P^T (bf - tf), one mother cell per wavefront.
template <int N, typename T>
__global__ void __launch_bounds__(256) k_mg_restrict(const T* __restrict__ bf, const T* __restrict__ tf,
                                                     T* __restrict__ bc, const T* __restrict__ etab, const XferCells g,
                                                     int64_t ncoarse, const int* stop) {
  using SH = XShape<N, T>;
  constexpr int N2 = SH::N2, N3 = SH::N3;
  __shared__ T s_tab[6 * N2];
  __shared__ T s_all[SH::WAVES * SH::SLICE];
  if (stop && *stop) return;
  for (int e = threadIdx.x; e < 6 * N2; e += blockDim.x) s_tab[e] = etab[e];
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t C = static_cast<int64_t>(blockIdx.x) * SH::WAVES + wave;
  if (C >= ncoarse) return;
  T* F = s_all + wave * SH::SLICE;      // nch N3: [sz][sy][sx][l][j][i]
  T* B = F + 8 * N3;                      // [sy][sx][c][j][i]
  T* A = B + 4 * N3;                      // [sx][c][b][i]
  const int CX = static_cast<int>(C % g.cnx);
  const int CY = static_cast<int>((C / g.cnx) % g.cny);
  const int CZ = static_cast<int>(C / (static_cast<int64_t>(g.cnx) * g.cny));
  const int rx = g.r[0], ry = g.r[1], rz = g.r[2];
  const int nch = rx * ry * rz;
  for (int e = lane; e < nch * N3; e += 64) {
    const int r = e % N3, ch = e / N3;
    const int sx = ch % rx, sy = (ch / rx) % ry, sz = ch / (rx * ry);
    const int64_t at = child_cell(g, CX, CY, CZ, sx, sy, sz) * N3 + r;
    F[e] = bf[at] - tf[at];
  }
  wave_sync();
  for (int e = lane; e < ry * rx * N3; e += 64) {      // B[sy][sx][c][j][i] = sum_{sz,l} Ez[sz][l][c] F[sz][sy][sx][l][j][i]
    const int ji = e % N2, c = (e / N2) % N, sx = (e / N3) % rx, sy = e / (rx * N3);
    T acc = 0;
    for (int sz = 0; sz < rz; ++sz) {
      const T* ez = s_tab + (2 * 2 + sz) * N2 + c;
      const T* src = F + ((sz * ry + sy) * rx + sx) * N3 + ji;
#pragma unroll
      for (int l = 0; l < N; ++l) acc = fma(ez[l * N], src[l * N2], acc);
    }
    B[e] = acc;
  }
  wave_sync();
  for (int e = lane; e < rx * N3; e += 64) {           // A[sx][c][b][i] = sum_{sy,j} Ey[sy][j][b] B[sy][sx][c][j][i]
    const int i = e % N, b = (e / N) % N, c = (e / N2) % N, sx = e / N3;
    T acc = 0;
    for (int sy = 0; sy < ry; ++sy) {
      const T* ey = s_tab + (1 * 2 + sy) * N2 + b;
      const T* src = B + (sy * rx + sx) * N3 + c * N2 + i;
#pragma unroll
      for (int j = 0; j < N; ++j) acc = fma(ey[j * N], src[j * N], acc);
    }
    A[e] = acc;
  }
  wave_sync();
  for (int e = lane; e < N3; e += 64) {                // out[c][b][a] = sum_{sx,i} Ex[sx][i][a] A[sx][c][b][i]
    const int a = e % N, cb = e / N;
    T acc = 0;
    for (int sx = 0; sx < rx; ++sx) {
      const T* ex = s_tab + (0 * 2 + sx) * N2 + a;
      const T* src = A + sx * N3 + cb * N;
#pragma unroll
      for (int i = 0; i < N; ++i) acc = fma(ex[i * N], src[i], acc);
    }
    bc[C * N3 + e] = acc;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_mg_cast_in(const double* __restrict__ r, T* __restrict__ b, int64_t N,
                                                    const int* stop) {
  if (stop && *stop) return;
  MG_GRID_STRIDE(i, N) b[i] = static_cast<T>(r[i]);
}

// x = s dinv b: the first Chebyshev iterate from zero
template <typename T>
__global__ void __launch_bounds__(256) k_mg_jacobi(const T* __restrict__ b, const T* __restrict__ dinv,
                                                   T* __restrict__ x, T s, int64_t N, const int* stop) {
  if (stop && *stop) return;
  MG_GRID_STRIDE(i, N) x[i] = s * dinv[i] * b[i];
}

// dst = xk + c1 (xk - dst) + c2 dinv (b - t), t = H xk (dst read as zero when prev_zero)
template <typename T>
__global__ void __launch_bounds__(256) k_mg_cheb_vec(const T* __restrict__ xk, T* __restrict__ dst,
                                                     const T* __restrict__ b, const T* __restrict__ t,
                                                     const T* __restrict__ dinv, T c1, T c2, int prev_zero, int64_t N,
                                                     const int* stop) {
  if (stop && *stop) return;
  MG_GRID_STRIDE(i, N) {
    const T x = xk[i], p = prev_zero ? T(0) : dst[i];
    dst[i] = fma(c2 * dinv[i], b[i] - t[i], fma(c1, x - p, x));
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_mg_cast_out(const T* __restrict__ x, double* __restrict__ z, int64_t N) {
  MG_GRID_STRIDE(i, N) z[i] = static_cast<double>(x[i]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_mg_diag(const double* __restrict__ diag, T* __restrict__ dinv,
                                                 T* __restrict__ dsq, int64_t N) {
  MG_GRID_STRIDE(i, N) {
    const double v = 1.0 / diag[i];
    dinv[i] = static_cast<T>(v);
    dsq[i] = static_cast<T>(sqrt(v));
  }
}

unsigned vec_grid(int64_t N) {
  const int64_t b = (N + 255) / 256;
  return static_cast<unsigned>(b < kMgVecBlocks ? (b > 0 ? b : 1) : kMgVecBlocks);
}

template <int N, typename T>
dgmf_status xfer_n(bool prolong, const MgXfer& x, const T* a, const T* b, T* out, const T* etab, const int* stop,
                   hipStream_t s) {
  using SH = XShape<N, T>;
  XferCells g{x.cnx, x.cny, x.cnz, x.fnx, x.fny, {x.r[0], x.r[1], x.r[2]}};
  const int64_t nc = static_cast<int64_t>(x.cnx) * x.cny * x.cnz;
  const int64_t blocks = (nc + SH::WAVES - 1) / SH::WAVES;
  if (blocks > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "multigrid: too many cells for one launch");
  if (prolong) {
    hipLaunchKernelGGL((k_mg_prolong<N, T>), dim3(static_cast<unsigned>(blocks)), dim3(64 * SH::WAVES), 0, s, a, out,
                       etab, g, nc, stop);
    DGMF_LAUNCH_CHECK("k_mg_prolong");
  } else {
    hipLaunchKernelGGL((k_mg_restrict<N, T>), dim3(static_cast<unsigned>(blocks)), dim3(64 * SH::WAVES), 0, s, a, b,
                       out, etab, g, nc, stop);
    DGMF_LAUNCH_CHECK("k_mg_restrict");
  }
  return DGMF_OK;
}

template <typename T>
dgmf_status xfer(int n, bool prolong, const MgXfer& x, const T* a, const T* b, T* out, const T* etab, const int* stop,
                 hipStream_t s) {
  switch (n) {
    case 2: return xfer_n<2, T>(prolong, x, a, b, out, etab, stop, s);
    case 3: return xfer_n<3, T>(prolong, x, a, b, out, etab, stop, s);
    case 4: return xfer_n<4, T>(prolong, x, a, b, out, etab, stop, s);
    case 5: return xfer_n<5, T>(prolong, x, a, b, out, etab, stop, s);
    case 6: return xfer_n<6, T>(prolong, x, a, b, out, etab, stop, s);
    case 7: return xfer_n<7, T>(prolong, x, a, b, out, etab, stop, s);
    case 8: return xfer_n<8, T>(prolong, x, a, b, out, etab, stop, s);
    default: return fail(DGMF_UNSUPPORTED, "multigrid: n = %d not built", n);
  }
}

}  // namespace

template <typename T>
dgmf_status launch_mg_prolong(int n, const MgXfer& x, const T* xc, T* xf, const T* etab, const int* stop,
                              hipStream_t s) {
  return xfer<T>(n, true, x, xc, nullptr, xf, etab, stop, s);
}

template <typename T>
dgmf_status launch_mg_restrict(int n, const MgXfer& x, const T* bf, const T* tf, T* bc, const T* etab,
                               const int* stop, hipStream_t s) {
  return xfer<T>(n, false, x, bf, tf, bc, etab, stop, s);
}

template <typename T>
dgmf_status launch_mg_cast_in(const double* r, T* b, int64_t N, const int* stop, hipStream_t s) {
  hipLaunchKernelGGL((k_mg_cast_in<T>), dim3(vec_grid(N)), dim3(256), 0, s, r, b, N, stop);
  DGMF_LAUNCH_CHECK("k_mg_cast_in");
  return DGMF_OK;
}

template <typename T>
dgmf_status launch_mg_cast_out(const T* x, double* z, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL((k_mg_cast_out<T>), dim3(vec_grid(N)), dim3(256), 0, s, x, z, N);
  DGMF_LAUNCH_CHECK("k_mg_cast_out");
  return DGMF_OK;
}

template <typename T>
dgmf_status launch_mg_jacobi(const T* b, const T* dinv, T* x, double scale, int64_t N, const int* stop,
                             hipStream_t s) {
  hipLaunchKernelGGL((k_mg_jacobi<T>), dim3(vec_grid(N)), dim3(256), 0, s, b, dinv, x, static_cast<T>(scale), N,
                     stop);
  DGMF_LAUNCH_CHECK("k_mg_jacobi");
  return DGMF_OK;
}

template <typename T>
dgmf_status launch_mg_cheb_vec(const T* xk, T* dst, const T* b, const T* t, const T* dinv, double c1, double c2,
                               bool prev_zero, int64_t N, const int* stop, hipStream_t s) {
  hipLaunchKernelGGL((k_mg_cheb_vec<T>), dim3(vec_grid(N)), dim3(256), 0, s, xk, dst, b, t, dinv, static_cast<T>(c1),
                     static_cast<T>(c2), prev_zero ? 1 : 0, N, stop);
  DGMF_LAUNCH_CHECK("k_mg_cheb_vec");
  return DGMF_OK;
}

template <typename T>
dgmf_status launch_mg_diag(const double* diag, T* dinv, T* dsq, int64_t N, hipStream_t s) {
  hipLaunchKernelGGL((k_mg_diag<T>), dim3(vec_grid(N)), dim3(256), 0, s, diag, dinv, dsq, N);
  DGMF_LAUNCH_CHECK("k_mg_diag");
  return DGMF_OK;
}

#define DGMF_MG_INST(T)                                                                                            \
  template dgmf_status launch_mg_prolong<T>(int, const MgXfer&, const T*, T*, const T*, const int*, hipStream_t);  \
  template dgmf_status launch_mg_restrict<T>(int, const MgXfer&, const T*, const T*, T*, const T*, const int*,     \
                                             hipStream_t);                                                         \
  template dgmf_status launch_mg_cast_in<T>(const double*, T*, int64_t, const int*, hipStream_t);                  \
  template dgmf_status launch_mg_cast_out<T>(const T*, double*, int64_t, hipStream_t);                             \
  template dgmf_status launch_mg_diag<T>(const double*, T*, T*, int64_t, hipStream_t);                          \
  template dgmf_status launch_mg_jacobi<T>(const T*, const T*, T*, double, int64_t, const int*, hipStream_t);     \
  template dgmf_status launch_mg_cheb_vec<T>(const T*, T*, const T*, const T*, const T*, double, double, bool,    \
                                             int64_t, const int*, hipStream_t);
DGMF_MG_INST(double)
DGMF_MG_INST(float)
#undef DGMF_MG_INST

}  // namespace dgmf
