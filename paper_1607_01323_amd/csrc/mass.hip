// The block-diagonal DG mass matrix and its inverse on affine hexahedra (gfx950).
//
// With the nodal basis on Gauss-Lobatto points the mass block of a cell is
// not diagonal (Sec. 5, implementation).  On an affine cell it is
//   M_K = |det J| (Mh (x) Mh (x) Mh),   Mh = S^T W S,
// S the square (n_q = k+1) node-to-Gauss-point interpolation and W the Gauss
// weights on [0,1].  Inverting the 1D factors one by one gives the tensorial
// inverse Mh^{-1} = S^{-1} W^{-1} S^{-T}, formed on the host in long double.
// Because |det J| is constant on an affine cell, the paper's
// transform / inverse-weight / transform sequence collapses into three 1D
// sweeps by Mh^{-1} and one scale by 1/|det J|.  The same kernel applies M
// itself (three sweeps by Mh and the scale |det J|).
//
// Layout: n^2 lanes per cell, 64/n^2 cells per wavefront, four independent
// wavefronts per workgroup (no workgroup barrier).  Lane (i, j) loads the
// z-line of its cell, applies the z sweep in registers and writes the result
// to the wavefront's LDS slice; the y and x sweeps work on whole lines in
// place there (one line per lane); the wavefront's cells are contiguous in
// memory and leave through one coalesced store.  Fields are consecutive
// blocks of n_cells cells, so several fields form one flat list of cells.
#include "internal.h"

namespace dgmf {
namespace {

template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N>
struct IMShape {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int CPW = 64 / N2;       // cells per wavefront
  static constexpr int CP = N3 | 1;         // LDS pitch of a cell (odd: spreads banks)
  static constexpr int WAVES = 4, THREADS = 64 * WAVES;
};

// INV: dst = M^{-1} src (table Mh^{-1}, scale jscale / (hx hy hz)); else
// dst = M src (table Mh, scale jscale hx hy hz).
template <int N, typename T, bool INV>
__global__ void __launch_bounds__(256) k_block_mass(const T* src, T* dst, const CartGeom<T> g, const T jscale,
                                                      const T* minv_g, const int64_t ncells, const int64_t total) {
  using SH = IMShape<N>;
  constexpr int N2 = SH::N2, N3 = SH::N3, CP = SH::CP, CPW = SH::CPW;
  __shared__ T s[SH::WAVES * CPW * CP];
  const cptr<T> Mi = (cptr<T>)minv_g;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t first = (static_cast<int64_t>(blockIdx.x) * SH::WAVES + wave) * CPW;
  if (first >= total) return;
  T* sw = s + wave * CPW * CP;
  const int cs = lane / N2, t = lane % N2;
  const int64_t fc = first + cs;
  const bool act = cs < CPW && fc < total;
  T* cell = sw + cs * CP;
  T v[N];
  if (act) {
    const T* in = src + fc * N3 + t;
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = in[m * N2];
#pragma unroll
    for (int l = 0; l < N; ++l) {
      T r = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) r = fma(Mi[l * N + m], v[m], r);
      cell[l * N2 + t] = r;
    }
  }
  wave_sync();
  if (act) {                                   // y lines: (i, l) = (t % N, t / N)
    T* p = cell + (t / N) * N2 + t % N;
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = p[m * N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T r = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) r = fma(Mi[j * N + m], v[m], r);
      p[j * N] = r;
    }
  }
  wave_sync();
  if (act) {                                   // x lines: (j, l), offset t * N
    const int64_t c = fc % ncells;
    const int cx = static_cast<int>(c % g.nx);
    const int64_t r2 = c / g.nx;
    const int cy = static_cast<int>(r2 % g.ny), cz = static_cast<int>(r2 / g.ny);
    const T sc = INV ? jscale * g.hinv[0][cx] * g.hinv[1][cy] * g.hinv[2][cz]
                     : jscale * g.h[0][cx] * g.h[1][cy] * g.h[2][cz];
    T* p = cell + t * N;
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = p[m];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T r = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) r = fma(Mi[i * N + m], v[m], r);
      p[i] = sc * r;
    }
  }
  wave_sync();
  const int64_t rem = total - first;
  const int nc = rem < CPW ? static_cast<int>(rem) : CPW;
  T* out = dst + first * N3;
  for (int e = lane; e < nc * N3; e += 64) out[e] = sw[(e / N3) * CP + e % N3];
}

// Curved cells (the Jacobian varies inside the cell): with m_q = w_q det J_q at
// the Gauss points (the stored metric's last cell entry),
//   M = S^T (x)3 diag(m) S (x)3,   M^{-1} = S^{-1} (x)3 diag(1/m) S^{-T} (x)3,
// i.e. the paper's tensorial inverse with the point weights between the two
// transforms: three sweeps by P, the pointwise scale, three sweeps by Q.
// tab: [S | S^T | S^{-T} | S^{-1}] (n x n each, row-major [out][in]); the
// mass uses (P, Q) = (S, S^T), the inverse (S^{-T}, S^{-1}).  Same lane layout as
// k_block_mass; m read per node from the stored metric of the cell.
template <int N, typename T, bool INV>
__global__ void __launch_bounds__(256) k_point_mass(const T* src, T* dst, const T* tab_g, const T* cm,
                                                      const int64_t ncells, const int64_t total) {
  using SH = IMShape<N>;
  constexpr int N2 = SH::N2, N3 = SH::N3, CP = SH::CP, CPW = SH::CPW;
  __shared__ T s[SH::WAVES * CPW * CP];
  const cptr<T> tab = (cptr<T>)tab_g;
  const cptr<T> P = tab + (INV ? 2 : 0) * N * N;
  const cptr<T> Q = tab + (INV ? 3 : 1) * N * N;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t first = (static_cast<int64_t>(blockIdx.x) * SH::WAVES + wave) * CPW;
  if (first >= total) return;
  T* sw = s + wave * CPW * CP;
  const int cs = lane / N2, t = lane % N2;
  const int64_t fc = first + cs;
  const bool act = cs < CPW && fc < total;
  T* cell = sw + cs * CP;
  T v[N];
  // along z (from memory), y, x by P; scale by m (or 1/m); along x, y, z by Q
  if (act) {
    const T* in = src + fc * N3 + t;
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = in[m * N2];
#pragma unroll
    for (int l = 0; l < N; ++l) {
      T r = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) r = fma(P[l * N + m], v[m], r);
      cell[l * N2 + t] = r;
    }
  }
  wave_sync();
  if (act) {
    T* p = cell + (t / N) * N2 + t % N;
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = p[m * N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T r = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) r = fma(P[j * N + m], v[m], r);
      p[j * N] = r;
    }
  }
  wave_sync();
  if (act) {                                   // x lines: (j, l), offset t * N; scale, then Q along x
    const T* mw = cm + (fc % ncells) * 7 * N3 + 6 * N3 + t * N;
    T* p = cell + t * N;
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = p[m];
    T u[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T r = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) r = fma(P[i * N + m], v[m], r);
      u[i] = INV ? r / mw[i] : r * mw[i];
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      T r = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) r = fma(Q[i * N + m], u[m], r);
      p[i] = r;
    }
  }
  wave_sync();
  if (act) {
    T* p = cell + (t / N) * N2 + t % N;
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = p[m * N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      T r = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) r = fma(Q[j * N + m], v[m], r);
      p[j * N] = r;
    }
  }
  wave_sync();
  if (act) {                                   // z lines, in place
    T* p = cell + t;
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = p[m * N2];
#pragma unroll
    for (int l = 0; l < N; ++l) {
      T r = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) r = fma(Q[l * N + m], v[m], r);
      p[l * N2] = r;
    }
  }
  wave_sync();
  const int64_t rem = total - first;
  const int nc = rem < CPW ? static_cast<int>(rem) : CPW;
  T* out = dst + first * N3;
  for (int e = lane; e < nc * N3; e += 64) out[e] = sw[(e / N3) * CP + e % N3];
}

template <int N, typename T>
dgmf_status launch_pn(const T* tab, const T* cm, const T* src, T* dst, int64_t ncells, int64_t total, bool inv,
                      hipStream_t s) {
  using SH = IMShape<N>;
  const int64_t waves = (total + SH::CPW - 1) / SH::CPW;
  const int64_t blocks = (waves + SH::WAVES - 1) / SH::WAVES;
  if (blocks > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "mass: too many cells for one launch");
  if (inv)
    hipLaunchKernelGGL((k_point_mass<N, T, true>), dim3(static_cast<unsigned>(blocks)), dim3(SH::THREADS), 0, s,
                       src, dst, tab, cm, ncells, total);
  else
    hipLaunchKernelGGL((k_point_mass<N, T, false>), dim3(static_cast<unsigned>(blocks)), dim3(SH::THREADS), 0, s,
                       src, dst, tab, cm, ncells, total);
  DGMF_LAUNCH_CHECK("k_point_mass");
  return DGMF_OK;
}

template <int N, typename T>
dgmf_status launch_n(const CartGeom<T>& g, T jscale, const T* minv, const T* src, T* dst, int64_t ncells,
                     int64_t total, bool inv, hipStream_t s) {
  using SH = IMShape<N>;
  const int64_t waves = (total + SH::CPW - 1) / SH::CPW;
  const int64_t blocks = (waves + SH::WAVES - 1) / SH::WAVES;
  if (blocks > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "inverse_mass: too many cells for one launch");
  if (inv)
    hipLaunchKernelGGL((k_block_mass<N, T, true>), dim3(static_cast<unsigned>(blocks)), dim3(SH::THREADS), 0, s,
                       src, dst, g, jscale, minv, ncells, total);
  else
    hipLaunchKernelGGL((k_block_mass<N, T, false>), dim3(static_cast<unsigned>(blocks)), dim3(SH::THREADS), 0, s,
                       src, dst, g, jscale, minv, ncells, total);
  DGMF_LAUNCH_CHECK("k_block_mass");
  return DGMF_OK;
}

}  // namespace

template <typename T>
dgmf_status launch_block_mass(int n, const CartGeom<T>& g, T jscale, const T* table, const T* src, T* dst,
                              int64_t ncells, int nfields, bool inverse, hipStream_t s) {
  const int64_t total = ncells * nfields;
  if (total == 0) return DGMF_OK;
  switch (n) {
    case 2: return launch_n<2, T>(g, jscale, table, src, dst, ncells, total, inverse, s);
    case 3: return launch_n<3, T>(g, jscale, table, src, dst, ncells, total, inverse, s);
    case 4: return launch_n<4, T>(g, jscale, table, src, dst, ncells, total, inverse, s);
    case 5: return launch_n<5, T>(g, jscale, table, src, dst, ncells, total, inverse, s);
    case 6: return launch_n<6, T>(g, jscale, table, src, dst, ncells, total, inverse, s);
    case 7: return launch_n<7, T>(g, jscale, table, src, dst, ncells, total, inverse, s);
    case 8: return launch_n<8, T>(g, jscale, table, src, dst, ncells, total, inverse, s);
    default: return fail(DGMF_UNSUPPORTED, "mass: n = %d not built", n);
  }
}

template <typename T>
dgmf_status launch_point_mass(int n, const T* tab, const T* cm, const T* src, T* dst, int64_t ncells, int nfields,
                              bool inverse, hipStream_t s) {
  const int64_t total = ncells * nfields;
  if (total == 0) return DGMF_OK;
  switch (n) {
    case 2: return launch_pn<2, T>(tab, cm, src, dst, ncells, total, inverse, s);
    case 3: return launch_pn<3, T>(tab, cm, src, dst, ncells, total, inverse, s);
    case 4: return launch_pn<4, T>(tab, cm, src, dst, ncells, total, inverse, s);
    case 5: return launch_pn<5, T>(tab, cm, src, dst, ncells, total, inverse, s);
    case 6: return launch_pn<6, T>(tab, cm, src, dst, ncells, total, inverse, s);
    case 7: return launch_pn<7, T>(tab, cm, src, dst, ncells, total, inverse, s);
    case 8: return launch_pn<8, T>(tab, cm, src, dst, ncells, total, inverse, s);
    default: return fail(DGMF_UNSUPPORTED, "mass: n = %d not built", n);
  }
}

template dgmf_status launch_point_mass<double>(int, const double*, const double*, const double*, double*, int64_t,
                                               int, bool, hipStream_t);
template dgmf_status launch_point_mass<float>(int, const float*, const float*, const float*, float*, int64_t, int,
                                              bool, hipStream_t);

template dgmf_status launch_block_mass<double>(int, const CartGeom<double>&, double, const double*, const double*,
                                               double*, int64_t, int, bool, hipStream_t);
template dgmf_status launch_block_mass<float>(int, const CartGeom<float>&, float, const float*, const float*, float*,
                                              int64_t, int, bool, hipStream_t);

}  // namespace dgmf
