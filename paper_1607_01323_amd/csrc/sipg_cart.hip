// Matrix-free SIPG Laplace / Helmholtz apply on axis-aligned hexahedra (gfx950).
//
// Operator (Sec. 3.2, pressure Poisson step and scalar viscous step; Sec. 5
// sum factorisation): H = mu M + nu A with the SIPG Laplacian A.  On a cell
// of size hx*hy*hz the Jacobian is constant and diagonal, so with n_q = k+1
// Gauss points (exact for every integrand here) each cell and face integral
// factorises into 1D reference matrices:
//   Mhat_ij = sum_q w_q l_i(x_q) l_j(x_q),  Khat_ij = sum_q w_q l_i'(x_q) l_j'(x_q),
// and the operator restricted to one cell's rows is
//   H u = (Mz x My)(A_x u) + (Mz x Mx)(A_y u) + (My x Mx)(A_z u),
// where A_d acts along the lines of direction d and contains the stiffness,
// the face fluxes of the two faces normal to d (neighbour lines enter there)
// and, for d = x, the mass term.  With GLL nodes the face value of a line is
// its end node, and the normal derivative is the end-point derivative row
// l'(0) or l'(1) applied to the line.
//
// Kernel layout: one workgroup per batch of CPB = 256 / n^2 cells, n^2
// threads per cell, each thread owning one line of its cell per pass.  The
// cell tensor and intermediates live in LDS with a padded line pitch n+1;
// neighbour lines are read straight from global memory (L2 / Infinity Cache
// hits: each cell is read by its six neighbours).  Six passes:
//   1 x-lines: a = A_x u                         (neighbour x-lines)
//   2 y-lines: f = A_y u, c = My a              (neighbour y-lines)
//   3 z-lines: g = A_z u                         (neighbour z-lines)
//   4 x-lines: c += Mx f, g = Mx g
//   5 y-lines: g = My g
//   6 z-lines: dst = Mz c + g                    (coalesced store)
#include "internal.h"

namespace dgmf {
namespace {

// gfx950 dispatches consecutive workgroups round-robin over its 8 XCDs, each
// with a private L2.  Remap so that every XCD walks a contiguous range of
// cells: the face neighbours a block reads are then mostly in its own L2.
constexpr int kXcds = 8;

__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t nblocks) {
  const int64_t q = nblocks / kXcds, rem = nblocks % kXcds;
  const int64_t x = b % kXcds, r = b / kXcds;
  return x * q + (x < rem ? x : rem) + r;
}

template <int N>
struct Shape {
  static constexpr int N2 = N * N;
  static constexpr int N3 = N2 * N;
  static constexpr int CPB = 256 / N2;        // cells per block
  static constexpr int P = N + 1;             // padded x-line pitch in LDS
  static constexpr int CL = N2 * P;           // LDS words per cell per buffer
};

template <int N, typename T>
__device__ __forceinline__ void matvec(const T* __restrict__ A, const T (&x)[N], T (&y)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = A[i * N] * x[0];
#pragma unroll
    for (int j = 1; j < N; ++j) s = fma(A[i * N + j], x[j], s);
    y[i] = s;
  }
}

// One direction's line operator A_d for one line of the cell.
//   u      : the line of this cell
//   ul, ur : the same line of the low / high neighbour (unused on Dirichlet faces)
//   sigma  : nu * (product of the two tangential cell sizes)
//   massc  : mu * cell volume (x direction only, else 0)
// Interior face on the high side ([u] = u_N-1 - ur_0, {{u'}} = (l'(1).u/h + l'(0).ur/hr)/2):
//   out_i += sigma (-1/2 l_i'(1)/h [u] + delta_{i,N-1} (-{{u'}} + tau [u]))
// Interior face on the low side ([u] = ul_N-1 - u_0, {{u'}} = (l'(1).ul/hl + l'(0).u/h)/2):
//   out_i += sigma (-1/2 l_i'(0)/h [u] + delta_{i,0} ({{u'}} - tau [u]))
// Dirichlet high face: out_i += sigma (-l_i'(1)/h u_N-1 + delta_{i,N-1}(-l'(1).u/h + 2 tau u_N-1))
// Dirichlet low face:  out_i += sigma ( l_i'(0)/h u_0   + delta_{i,0}  ( l'(0).u/h + 2 tau u_0))
template <int N, typename T>
__device__ __forceinline__ void sipg_line(const T* __restrict__ tab, const T (&u)[N], const T (&ul)[N],
                                          const T (&ur)[N], bool dirL, bool dirR, T hinv, T hlinv, T hrinv,
                                          T tauL, T tauR, T sigma, T massc, T (&out)[N]) {
  const T* Mh = tab;
  const T* Kh = tab + N * N;
  const T* g0 = tab + 2 * N * N;
  const T* g1 = g0 + N;
  T gu0 = 0, gu1 = 0;
#pragma unroll
  for (int m = 0; m < N; ++m) {
    gu0 = fma(g0[m], u[m], gu0);
    gu1 = fma(g1[m], u[m], gu1);
  }
  gu0 *= hinv;
  gu1 *= hinv;
  T jr, cr, jl, cl;
  if (dirR) {
    jr = u[N - 1];
    cr = -gu1 + T(2) * tauR * u[N - 1];
  } else {
    T gr = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) gr = fma(g0[m], ur[m], gr);
    const T jump = u[N - 1] - ur[0];
    const T avg = T(0.5) * (gu1 + gr * hrinv);
    jr = T(0.5) * jump;
    cr = -avg + tauR * jump;
  }
  if (dirL) {
    jl = u[0];
    cl = gu0 + T(2) * tauL * u[0];
  } else {
    T gl = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) gl = fma(g1[m], ul[m], gl);
    const T jump = ul[N - 1] - u[0];
    const T avg = T(0.5) * (gl * hlinv + gu0);
    jl = T(-0.5) * jump;
    cl = avg - tauL * jump;
  }
  T ku[N];
  matvec<N, T>(Kh, u, ku);
  const T sk = sigma * hinv;
  const T sjr = sigma * hinv * jr, sjl = sigma * hinv * jl;
#pragma unroll
  for (int i = 0; i < N; ++i) out[i] = fma(sk, ku[i], fma(-g1[i], sjr, g0[i] * sjl));
  out[N - 1] = fma(sigma, cr, out[N - 1]);
  out[0] = fma(sigma, cl, out[0]);
  if (massc != T(0)) {
    T mu_[N];
    matvec<N, T>(Mh, u, mu_);
#pragma unroll
    for (int i = 0; i < N; ++i) out[i] = fma(massc, mu_[i], out[i]);
  }
}

template <typename T>
struct CellInfo {
  int c[3];      // cell coordinates
  T h[3], hinv[3], tp[3];
  T tau;         // tau_e of this cell
};

template <typename T>
__device__ __forceinline__ void cell_info(const CartGeom<T>& g, int64_t cell, CellInfo<T>& ci) {
  ci.c[0] = static_cast<int>(cell % g.nx);
  const int64_t r = cell / g.nx;
  ci.c[1] = static_cast<int>(r % g.ny);
  ci.c[2] = static_cast<int>(r / g.ny);
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    ci.h[d] = g.h[d][ci.c[d]];
    ci.hinv[d] = g.hinv[d][ci.c[d]];
    ci.tp[d] = g.tp[d][ci.c[d]];
  }
  ci.tau = g.pen * (ci.tp[0] + ci.tp[1] + ci.tp[2]);
}

// Neighbour across the low (side 0) or high (side 1) face in direction d.
// Returns false on a Dirichlet face.  Fills the neighbour's cell index, 1/h and
// the face penalty tau_F = max(tau_e, tau_e').
template <typename T>
__device__ __forceinline__ bool neighbour(const CartGeom<T>& g, const CellInfo<T>& ci, int64_t cell, int d,
                                          int side, int64_t& nb, T& nhinv, T& tauF) {
  const int nd = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
  int cc = ci.c[d] + (side ? 1 : -1);
  if (cc < 0 || cc >= nd) {
    if (!g.per[d]) {
      tauF = ci.tau;
      return false;
    }
    cc = cc < 0 ? nd - 1 : 0;
  }
  const int64_t stride = d == 0 ? 1 : (d == 1 ? g.nx : static_cast<int64_t>(g.nx) * g.ny);
  nb = cell + static_cast<int64_t>(cc - ci.c[d]) * stride;
  nhinv = g.hinv[d][cc];
  const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
  const T taun = g.pen * (g.tp[d][cc] + ci.tp[d1] + ci.tp[d2]);
  tauF = ci.tau > taun ? ci.tau : taun;
  return true;
}

template <int N, typename T>
__device__ __forceinline__ void load_line(const T* __restrict__ base, int stride, T (&v)[N]) {
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] = base[m * stride];
}

// Apply A_d to the line of this cell that starts at element offset `off`
// (element stride `stride` inside a cell), reading own values from LDS.
template <int N, typename T>
__device__ __forceinline__ void dir_op(const CartGeom<T>& g, const T* __restrict__ src, const CellInfo<T>& ci,
                                       int64_t cell, int d, const T (&u)[N], int goff, int gstride, T massc,
                                       T (&out)[N]) {
  constexpr int N3 = N * N * N;
  T ul[N], ur[N];
  int64_t nb;
  T hl = 0, hr = 0, tauL, tauR;
  const bool hasL = neighbour(g, ci, cell, d, 0, nb, hl, tauL);
  if (hasL) load_line<N, T>(src + nb * N3 + goff, gstride, ul);
  const bool hasR = neighbour(g, ci, cell, d, 1, nb, hr, tauR);
  if (hasR) load_line<N, T>(src + nb * N3 + goff, gstride, ur);
  const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
  const T sigma = g.nu * ci.h[d1] * ci.h[d2];
  sipg_line<N, T>(g.tab, u, ul, ur, !hasL, !hasR, ci.hinv[d], hl, hr, tauL, tauR, sigma, massc, out);
}

template <int N, typename T>
__global__ void __launch_bounds__(256) k_sipg_cart_apply(const T* __restrict__ src, T* __restrict__ dst,
                                                         const CartGeom<T> g, int64_t ncells,
                                                         double* __restrict__ partials, const int* stop) {
  if (stop && *stop) return;   // uniform for the whole grid: CG already finished
  using S = Shape<N>;
  constexpr int N2 = S::N2, N3 = S::N3, P = S::P, CL = S::CL, CPB = S::CPB;
  __shared__ T s_u[CPB * CL];
  __shared__ T s_a[CPB * CL];
  __shared__ T s_b[CPB * CL];
  __shared__ double s_red[3 * (256 / 64)];

  const int tid = threadIdx.x;
  const int lc = tid / N2;
  const int t = tid - lc * N2;
  const int t0 = t % N, t1 = t / N;
  const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
  const int64_t cell = blk * CPB + lc;
  const bool act = lc < CPB && cell < ncells;
  T* su = s_u + (lc < CPB ? lc : 0) * CL;
  T* sa = s_a + (lc < CPB ? lc : 0) * CL;
  T* sb = s_b + (lc < CPB ? lc : 0) * CL;
  CellInfo<T> ci;
  if (act) cell_info(g, cell, ci);
  const T* cs = src + (act ? cell : 0) * N3;

  // pass 1: x-lines (j, l) = (t0, t1)
  if (act) {
    const int j = t0, l = t1;
    T u[N], out[N];
    load_line<N, T>(cs + (l * N + j) * N, 1, u);
    dir_op<N, T>(g, src, ci, cell, 0, u, (l * N + j) * N, 1, g.mu * ci.h[0] * ci.h[1] * ci.h[2], out);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      su[(l * N + j) * P + i] = u[i];
      sa[(l * N + j) * P + i] = out[i];
    }
  }
  __syncthreads();
  // pass 2: y-lines (i, l) = (t0, t1): f = A_y u -> sb, c = My a -> sa
  if (act) {
    const int i = t0, l = t1;
    T u[N], f[N], a[N], c[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      u[j] = su[(l * N + j) * P + i];
      a[j] = sa[(l * N + j) * P + i];
    }
    dir_op<N, T>(g, src, ci, cell, 1, u, l * N2 + i, N, T(0), f);
    matvec<N, T>(g.tab, a, c);
#pragma unroll
    for (int j = 0; j < N; ++j) {
      sa[(l * N + j) * P + i] = c[j];
      sb[(l * N + j) * P + i] = f[j];
    }
  }
  __syncthreads();
  // pass 3: z-lines (i, j) = (t0, t1): g = A_z u -> su (in place)
  if (act) {
    const int i = t0, j = t1;
    T u[N], o[N];
#pragma unroll
    for (int l = 0; l < N; ++l) u[l] = su[(l * N + j) * P + i];
    dir_op<N, T>(g, src, ci, cell, 2, u, j * N + i, N2, T(0), o);
#pragma unroll
    for (int l = 0; l < N; ++l) su[(l * N + j) * P + i] = o[l];
  }
  __syncthreads();
  // pass 4: x-lines: c += Mx f (sa), g = Mx g (su)
  if (act) {
    const int j = t0, l = t1;
    T f[N], gg[N], c[N], r1[N], r2[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      f[i] = sb[(l * N + j) * P + i];
      gg[i] = su[(l * N + j) * P + i];
      c[i] = sa[(l * N + j) * P + i];
    }
    matvec<N, T>(g.tab, f, r1);
    matvec<N, T>(g.tab, gg, r2);
#pragma unroll
    for (int i = 0; i < N; ++i) {
      sa[(l * N + j) * P + i] = c[i] + r1[i];
      su[(l * N + j) * P + i] = r2[i];
    }
  }
  __syncthreads();
  // pass 5: y-lines: g = My g
  if (act) {
    const int i = t0, l = t1;
    T gg[N], r[N];
#pragma unroll
    for (int j = 0; j < N; ++j) gg[j] = su[(l * N + j) * P + i];
    matvec<N, T>(g.tab, gg, r);
#pragma unroll
    for (int j = 0; j < N; ++j) su[(l * N + j) * P + i] = r[j];
  }
  __syncthreads();
  // pass 6: z-lines: dst = Mz c + g
  double pq = 0.0, sq = 0.0, sp = 0.0;
  if (act) {
    const int i = t0, j = t1;
    T c[N], r[N];
#pragma unroll
    for (int l = 0; l < N; ++l) c[l] = sa[(l * N + j) * P + i];
    matvec<N, T>(g.tab, c, r);
    T* cd = dst + cell * N3;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const T v = r[l] + su[(l * N + j) * P + i];
      cd[(l * N + j) * N + i] = v;
      if (partials) {
        const double pv = static_cast<double>(cs[(l * N + j) * N + i]);
        pq += pv * static_cast<double>(v);
        sq += static_cast<double>(v);
        sp += pv;
      }
    }
  }
  if (partials) {
    // wave64 shuffle reduction, then across the block's waves
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      pq += __shfl_down(pq, o, 64);
      sq += __shfl_down(sq, o, 64);
      sp += __shfl_down(sp, o, 64);
    }
    const int w = tid >> 6;
    if ((tid & 63) == 0) {
      s_red[3 * w] = pq;
      s_red[3 * w + 1] = sq;
      s_red[3 * w + 2] = sp;
    }
    __syncthreads();
    if (tid == 0) {
      const int nw = blockDim.x >> 6;
      double a = 0, b = 0, c = 0;
      for (int k = 0; k < nw; ++k) {
        a += s_red[3 * k];
        b += s_red[3 * k + 1];
        c += s_red[3 * k + 2];
      }
      partials[4 * blk] = a;
      partials[4 * blk + 1] = b;
      partials[4 * blk + 2] = c;
    }
  }
}

// Diagonal: for each direction the diagonal of the line operator A_d (the
// own-line part, plus the neighbour-coupling part when a periodic direction
// has a single cell, so that the neighbour is the cell itself), obtained by
// applying A_d to unit vectors; then diag = Dx_i My_jj Mz_ll + ... .
template <int N, typename T>
__global__ void __launch_bounds__(256) k_sipg_cart_diag(T* __restrict__ diag, const CartGeom<T> g,
                                                        int64_t ncells) {
  constexpr int N2 = N * N, N3 = N2 * N;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= ncells * N3) return;
  const int64_t cell = gid / N3;
  const int loc = static_cast<int>(gid - cell * N3);
  const int idx[3] = {loc % N, (loc / N) % N, loc / N2};
  CellInfo<T> ci;
  cell_info(g, cell, ci);
  T dd[3], md[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int p = idx[d];
    md[d] = g.tab[p * N + p];
    T e[N], el[N], er[N], out[N];
    int64_t nb;
    T hl = 0, hr = 0, tauL, tauR;
    const bool hasL = neighbour(g, ci, cell, d, 0, nb, hl, tauL);
    const bool selfL = hasL && nb == cell;
    const bool hasR = neighbour(g, ci, cell, d, 1, nb, hr, tauR);
    const bool selfR = hasR && nb == cell;
#pragma unroll
    for (int m = 0; m < N; ++m) {
      e[m] = (m == p) ? T(1) : T(0);
      el[m] = selfL ? e[m] : T(0);
      er[m] = selfR ? e[m] : T(0);
    }
    const int d1 = d == 0 ? 1 : 0, d2 = d == 2 ? 1 : 2;
    const T sigma = g.nu * ci.h[d1] * ci.h[d2];
    const T massc = d == 0 ? g.mu * ci.h[0] * ci.h[1] * ci.h[2] : T(0);
    sipg_line<N, T>(g.tab, e, el, er, !hasL, !hasR, ci.hinv[d], hl, hr, tauL, tauR, sigma, massc, out);
    T v = out[0];
#pragma unroll
    for (int m = 1; m < N; ++m) v = (m == p) ? out[m] : v;
    dd[d] = v;
  }
  diag[gid] = dd[0] * md[1] * md[2] + md[0] * dd[1] * md[2] + md[0] * md[1] * dd[2];
}

template <int N, typename T>
dgmf_status launch_apply_n(const CartGeom<T>& g, const T* src, T* dst, int64_t ncells, double* partials,
                           const int* stop, hipStream_t s) {
  using S = Shape<N>;
  const int64_t blocks = (ncells + S::CPB - 1) / S::CPB;
  if (blocks > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "mesh too large for one launch");
  hipLaunchKernelGGL((k_sipg_cart_apply<N, T>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s,
                     src, dst, g, ncells, partials, stop);
  DGMF_LAUNCH_CHECK("k_sipg_cart_apply");
  return DGMF_OK;
}

template <int N, typename T>
dgmf_status launch_diag_n(const CartGeom<T>& g, T* diag, int64_t ncells, hipStream_t s) {
  const int64_t total = ncells * N * N * N;
  const int64_t blocks = (total + 255) / 256;
  hipLaunchKernelGGL((k_sipg_cart_diag<N, T>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, diag, g,
                     ncells);
  DGMF_LAUNCH_CHECK("k_sipg_cart_diag");
  return DGMF_OK;
}

}  // namespace

int sipg_cart_blocks(int n, int64_t ncells) {
  const int cpb = 256 / (n * n);
  return static_cast<int>((ncells + cpb - 1) / cpb);
}

template <typename T>
dgmf_status launch_sipg_cart_apply(int n, const CartGeom<T>& g, const T* src, T* dst, int64_t ncells,
                                   double* partials, const int* stop, hipStream_t s) {
  switch (n) {
    case 2: return launch_apply_n<2, T>(g, src, dst, ncells, partials, stop, s);
    case 3: return launch_apply_n<3, T>(g, src, dst, ncells, partials, stop, s);
    case 4: return launch_apply_n<4, T>(g, src, dst, ncells, partials, stop, s);
    case 5: return launch_apply_n<5, T>(g, src, dst, ncells, partials, stop, s);
    case 6: return launch_apply_n<6, T>(g, src, dst, ncells, partials, stop, s);
    case 7: return launch_apply_n<7, T>(g, src, dst, ncells, partials, stop, s);
    case 8: return launch_apply_n<8, T>(g, src, dst, ncells, partials, stop, s);
    default: return fail(DGMF_UNSUPPORTED, "degree %d not built", n - 1);
  }
}

template <typename T>
dgmf_status launch_sipg_cart_diag(int n, const CartGeom<T>& g, T* diag, int64_t ncells, hipStream_t s) {
  switch (n) {
    case 2: return launch_diag_n<2, T>(g, diag, ncells, s);
    case 3: return launch_diag_n<3, T>(g, diag, ncells, s);
    case 4: return launch_diag_n<4, T>(g, diag, ncells, s);
    case 5: return launch_diag_n<5, T>(g, diag, ncells, s);
    case 6: return launch_diag_n<6, T>(g, diag, ncells, s);
    case 7: return launch_diag_n<7, T>(g, diag, ncells, s);
    case 8: return launch_diag_n<8, T>(g, diag, ncells, s);
    default: return fail(DGMF_UNSUPPORTED, "degree %d not built", n - 1);
  }
}

template dgmf_status launch_sipg_cart_apply<double>(int, const CartGeom<double>&, const double*, double*, int64_t,
                                                    double*, const int*, hipStream_t);
template dgmf_status launch_sipg_cart_apply<float>(int, const CartGeom<float>&, const float*, float*, int64_t,
                                                   double*, const int*, hipStream_t);
template dgmf_status launch_sipg_cart_diag<double>(int, const CartGeom<double>&, double*, int64_t, hipStream_t);
template dgmf_status launch_sipg_cart_diag<float>(int, const CartGeom<float>&, float*, int64_t, hipStream_t);

}  // namespace dgmf
