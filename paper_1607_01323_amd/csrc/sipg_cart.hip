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
// Kernel layout: one workgroup per batch of CPB = 128 / n^2 cells, n^2
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

constexpr int kApplyThreads = 128;   // threads per workgroup of the apply kernel

template <int N>
struct Shape {
  static constexpr int N2 = N * N;
  static constexpr int N3 = N2 * N;
  static constexpr int CPB = (kApplyThreads / N2) > 0 ? kApplyThreads / N2 : 1;   // cells per block
  static constexpr int P = (N % 2) ? N : N + 1;   // odd x-line pitch in LDS: conflict-free x-line access
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

// ---------------------------------------------------------------- apply ---
// Traversal order: the mesh is cut into y-strips, one per XCD when ny >= 8
// (workgroup b runs on XCD b % 8), and each strip is walked z-major, then y,
// then x.  The z-neighbour layer a workgroup reads was written a strip layer
// earlier (nx * ny/8 cells), so it is still in that XCD's L2.
__host__ __device__ inline int strip_count(int ny) { return ny >= 8 ? 8 : 1; }

// out = smain (mat u) [+ massc (Mhat u)] + the two face fluxes of this line.
// ul / ur: the same line of the low / high neighbour (ignored on Dirichlet faces).
template <int N, typename T, bool MASS>
__device__ __forceinline__ void line_apply(const T* __restrict__ tab, const T* __restrict__ mat, T smain, T massc,
                                           const T (&u)[N], const T (&ul)[N], const T (&ur)[N], bool dirL,
                                           bool dirR, T hinv, T hlinv, T hrinv, T tauL, T tauR, T sigma,
                                           T (&out)[N]) {
  const T* g0 = tab + 2 * N * N;
  const T* g1 = g0 + N;
  T gu0 = g0[0] * u[0], gu1 = g1[0] * u[0];
#pragma unroll
  for (int m = 1; m < N; ++m) {
    gu0 = fma(g0[m], u[m], gu0);
    gu1 = fma(g1[m], u[m], gu1);
  }
  gu0 *= hinv;
  gu1 *= hinv;
  const T sh = sigma * hinv;
  T cR, eR, cL, eL;   // coefficients of l'(1)_i and l'(0)_i, and the end-node terms
  if (dirR) {
    cR = -sh * u[N - 1];
    eR = sigma * fma(T(2) * tauR, u[N - 1], -gu1);
  } else {
    T gr = g0[0] * ur[0];
#pragma unroll
    for (int m = 1; m < N; ++m) gr = fma(g0[m], ur[m], gr);
    const T jump = u[N - 1] - ur[0];
    const T avg = T(0.5) * fma(gr, hrinv, gu1);
    cR = T(-0.5) * sh * jump;
    eR = sigma * fma(tauR, jump, -avg);
  }
  if (dirL) {
    cL = sh * u[0];
    eL = sigma * fma(T(2) * tauL, u[0], gu0);
  } else {
    T gl = g1[0] * ul[0];
#pragma unroll
    for (int m = 1; m < N; ++m) gl = fma(g1[m], ul[m], gl);
    const T jump = ul[N - 1] - u[0];
    const T avg = T(0.5) * fma(gl, hlinv, gu0);
    cL = T(-0.5) * sh * jump;
    eL = sigma * fma(-tauL, jump, avg);
  }
  T us[N], um[N];
#pragma unroll
  for (int m = 0; m < N; ++m) {
    us[m] = smain * u[m];
    if (MASS) um[m] = massc * u[m];
  }
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = fma(cL, g0[i], cR * g1[i]);
#pragma unroll
    for (int m = 0; m < N; ++m) acc = fma(mat[i * N + m], us[m], acc);
    if (MASS) {
#pragma unroll
      for (int m = 0; m < N; ++m) acc = fma(tab[i * N + m], um[m], acc);
    }
    out[i] = acc;
  }
  out[0] += eL;
  out[N - 1] += eR;
}

// y = A x + c (c optional: accumulate into y's initial value)
template <int N, typename T>
__device__ __forceinline__ void matvec_acc(const T* __restrict__ A, const T (&x)[N], T (&y)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = y[i];
#pragma unroll
    for (int j = 0; j < N; ++j) s = fma(A[i * N + j], x[j], s);
    y[i] = s;
  }
}

template <int N, typename T, bool PER>
struct Nb {
  int idx;       // neighbour cell
  T hinv, tau;   // its 1/h along d and the face penalty
  bool dir;      // Dirichlet face
};

// Low (side 0) / high (side 1) neighbour along d of a cell at coordinate cd.
template <int N, typename T, bool PER>
__device__ __forceinline__ Nb<N, T, PER> nbr(const CartGeom<T>& g, int cell, int cd, int nd, int stride, int d,
                                             int side, T tau_c, T tp_other) {
  Nb<N, T, PER> r;
  int cn = cd + (side ? 1 : -1);
  r.dir = false;
  if (cn < 0 || cn >= nd) {
    if (!PER && !g.per[d]) {
      r.dir = true;
      r.idx = cell;
      r.hinv = T(0);
      r.tau = tau_c;
      return r;
    }
    cn = cn < 0 ? nd - 1 : 0;
  }
  r.idx = cell + (cn - cd) * stride;
  r.hinv = g.hinv[d][cn];
  const T tn = g.pen * (g.tp[d][cn] + tp_other);
  r.tau = tau_c > tn ? tau_c : tn;
  return r;
}

// w += s [ hinv (Mhat^-1 Khat u) + Mhat^-1 (face fluxes of this line) ]: one
// direction's line operator, premultiplied by the inverse 1D mass matrix.
// Face fluxes (unit tangential area): interior high face, [u] = u_N-1 - ur_0,
// {{u'}} = (l'(1).u/h + l'(0).ur/hr)/2:
//   -1/2 l'(1)_i/h [u] + delta_{i,N-1} (tau [u] - {{u'}});
// interior low face, [u] = ul_N-1 - u_0, {{u'}} = (l'(1).ul/hl + l'(0).u/h)/2:
//   -1/2 l'(0)_i/h [u] + delta_{i,0} ({{u'}} - tau [u]);
// Dirichlet faces mirror these with [u] = u and the boundary penalty 2 tau.
template <int N, typename T>
__device__ __forceinline__ void bline(const T* __restrict__ tab, const T (&u)[N], const T (&ul)[N],
                                      const T (&ur)[N], bool dirL, bool dirR, T hinv, T hlinv, T hrinv, T tauL,
                                      T tauR, T s, T (&w)[N]) {
  constexpr TabLayout L{N, N};
  const T* g0 = tab + L.g0();
  const T* g1 = tab + L.g1();
  const T* Kt = tab + L.ktil();
  const T* g0t = tab + L.g0t();
  const T* g1t = tab + L.g1t();
  const T* e0t = tab + L.e0t();
  const T* e1t = tab + L.e1t();
  T gu0 = g0[0] * u[0], gu1 = g1[0] * u[0];
#pragma unroll
  for (int m = 1; m < N; ++m) {
    gu0 = fma(g0[m], u[m], gu0);
    gu1 = fma(g1[m], u[m], gu1);
  }
  gu0 *= hinv;
  gu1 *= hinv;
  T cR, eR, cL, eL;
  if (dirR) {
    cR = -hinv * u[N - 1];
    eR = fma(T(2) * tauR, u[N - 1], -gu1);
  } else {
    T gr = g0[0] * ur[0];
#pragma unroll
    for (int m = 1; m < N; ++m) gr = fma(g0[m], ur[m], gr);
    const T jump = u[N - 1] - ur[0];
    const T avg = T(0.5) * fma(gr, hrinv, gu1);
    cR = T(-0.5) * hinv * jump;
    eR = fma(tauR, jump, -avg);
  }
  if (dirL) {
    cL = hinv * u[0];
    eL = fma(T(2) * tauL, u[0], gu0);
  } else {
    T gl = g1[0] * ul[0];
#pragma unroll
    for (int m = 1; m < N; ++m) gl = fma(g1[m], ul[m], gl);
    const T jump = ul[N - 1] - u[0];
    const T avg = T(0.5) * fma(gl, hlinv, gu0);
    cL = T(-0.5) * hinv * jump;
    eL = fma(-tauL, jump, avg);
  }
  const T sh = s * hinv;
  cR *= s;
  cL *= s;
  eR *= s;
  eL *= s;
  T us[N];
#pragma unroll
  for (int m = 0; m < N; ++m) us[m] = sh * u[m];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = fma(cR, g1t[i], fma(cL, g0t[i], fma(eR, e1t[i], fma(eL, e0t[i], w[i]))));
#pragma unroll
    for (int m = 0; m < N; ++m) acc = fma(Kt[i * N + m], us[m], acc);
    w[i] = acc;
  }
}

// The operator in factored form: with V = hx hy hz and Mhat the 1D mass matrix,
//   H u = V (Mz x My x Mx) ( mu u + sum_d (nu/h_d) Mhat^-1 A_d u ),
// A_d the line operator of direction d (stiffness and the fluxes of its two
// faces).  Five passes, each thread owning one line of its cell per pass:
//   1 z-lines: load u (coalesced), w = mu V u + B_z u   (z-neighbour lines)
//   2 y-lines: w += B_y u                              (y-neighbour lines)
//   3 x-lines: w += B_x u; w = Mx w                    (x-neighbours from LDS in-block)
//   4 y-lines: w = My w
//   5 z-lines: dst = Mz w                               (coalesced store)
template <int N, typename T, bool PER>
__global__ void __launch_bounds__(kApplyThreads) k_sipg_cart_apply(const T* __restrict__ src, T* __restrict__ dst,
                                                         const CartGeom<T> g, double* __restrict__ partials,
                                                         const int* stop) {
  if (stop && *stop) return;   // uniform for the whole grid: CG already finished
  using S = Shape<N>;
  constexpr int N2 = S::N2, N3 = S::N3, P = S::P, CL = S::CL, CPB = S::CPB;
  __shared__ T s_u[CPB * CL];
  __shared__ T s_w[CPB * CL];
  __shared__ double s_red[3 * (kApplyThreads / 64)];

  const int tid = threadIdx.x;
  const int lc = tid / N2;
  const int t = tid - lc * N2;
  const int t0 = t % N, t1 = t / N;
  // strip decomposition of the block index
  const int nstrip = strip_count(g.ny);
  const int sidx = blockIdx.x % nstrip, r = blockIdx.x / nstrip;
  const int base = g.ny / nstrip, extra = g.ny % nstrip;
  const int hs = base + (sidx < extra ? 1 : 0);
  const int ys = sidx * base + (sidx < extra ? sidx : extra);
  const int ncs = g.nx * hs * g.nz;
  const int q = r * CPB + lc;
  const bool act = lc < CPB && q < ncs;
  int c[3] = {0, 0, 0}, cell = 0;
  if (act) {
    c[0] = q % g.nx;
    const int tq = q / g.nx;
    c[1] = ys + tq % hs;
    c[2] = tq / hs;
    cell = (c[2] * g.ny + c[1]) * g.nx + c[0];
  }
  const int nd[3] = {g.nx, g.ny, g.nz};
  const int stride[3] = {1, g.nx, g.nx * g.ny};
  const int slot = (lc < CPB ? lc : 0) * CL;
  T* su = s_u + slot;
  T* sw = s_w + slot;
  T h[3], hinv[3], tp[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    h[d] = g.h[d][c[d]];
    hinv[d] = g.hinv[d][c[d]];
    tp[d] = g.tp[d][c[d]];
  }
  const T tau_c = g.pen * (tp[0] + tp[1] + tp[2]);
  const T vol = h[0] * h[1] * h[2];
  const T vnu = vol * g.nu;
  const T* Mh = g.tab;

  // pass 1: z-lines (i, j) = (t0, t1)
  T u[N];
  if (act) {
    const int off = t1 * N + t0;
    const Nb<N, T, PER> L = nbr<N, T, PER>(g, cell, c[2], nd[2], stride[2], 2, 0, tau_c, tp[0] + tp[1]);
    const Nb<N, T, PER> R = nbr<N, T, PER>(g, cell, c[2], nd[2], stride[2], 2, 1, tau_c, tp[0] + tp[1]);
    T zl[N], zr[N], w[N];
#pragma unroll
    for (int l = 0; l < N; ++l) {
      u[l] = src[cell * N3 + off + l * N2];
      zl[l] = L.dir ? T(0) : src[L.idx * N3 + off + l * N2];
      zr[l] = R.dir ? T(0) : src[R.idx * N3 + off + l * N2];
    }
    const T mv = g.mu * vol;
#pragma unroll
    for (int l = 0; l < N; ++l) w[l] = mv * u[l];
    bline<N, T>(g.tab, u, zl, zr, L.dir, R.dir, hinv[2], L.hinv, R.hinv, L.tau, R.tau, vnu * hinv[2], w);
#pragma unroll
    for (int l = 0; l < N; ++l) {
      su[(l * N + t1) * P + t0] = u[l];
      sw[(l * N + t1) * P + t0] = w[l];
    }
  }
  __syncthreads();
  // pass 2: y-lines (i, l) = (t0, t1)
  if (act) {
    const int i = t0, l = t1;
    const Nb<N, T, PER> L = nbr<N, T, PER>(g, cell, c[1], nd[1], stride[1], 1, 0, tau_c, tp[0] + tp[2]);
    const Nb<N, T, PER> R = nbr<N, T, PER>(g, cell, c[1], nd[1], stride[1], 1, 1, tau_c, tp[0] + tp[2]);
    T uy[N], yl[N], yr[N], w[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      yl[j] = L.dir ? T(0) : src[L.idx * N3 + l * N2 + j * N + i];
      yr[j] = R.dir ? T(0) : src[R.idx * N3 + l * N2 + j * N + i];
      uy[j] = su[(l * N + j) * P + i];
      w[j] = sw[(l * N + j) * P + i];
    }
    bline<N, T>(g.tab, uy, yl, yr, L.dir, R.dir, hinv[1], L.hinv, R.hinv, L.tau, R.tau, vnu * hinv[1], w);
#pragma unroll
    for (int j = 0; j < N; ++j) sw[(l * N + j) * P + i] = w[j];
  }
  __syncthreads();
  // pass 3: x-lines (j, l) = (t0, t1); x-neighbour lines from LDS when in this block
  if (act) {
    const Nb<N, T, PER> L = nbr<N, T, PER>(g, cell, c[0], nd[0], stride[0], 0, 0, tau_c, tp[1] + tp[2]);
    const Nb<N, T, PER> R = nbr<N, T, PER>(g, cell, c[0], nd[0], stride[0], 0, 1, tau_c, tp[1] + tp[2]);
    const int lo = (t1 * N + t0) * P;
    const int sl_l = lc + (c[0] > 0 ? -1 : g.nx - 1);
    const int sl_r = lc + (c[0] < g.nx - 1 ? 1 : 1 - g.nx);
    const bool inl = sl_l >= 0 && sl_l < CPB && q + (sl_l - lc) < ncs;
    const bool inr = sl_r >= 0 && sl_r < CPB && q + (sl_r - lc) < ncs;
    const int offx = (t1 * N + t0) * N;
    T ux[N], xl[N], xr[N], w[N], o[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      ux[i] = su[lo + i];
      w[i] = sw[lo + i];
      xl[i] = L.dir ? T(0) : (inl ? s_u[sl_l * CL + lo + i] : src[L.idx * N3 + offx + i]);
      xr[i] = R.dir ? T(0) : (inr ? s_u[sl_r * CL + lo + i] : src[R.idx * N3 + offx + i]);
      o[i] = T(0);
    }
    bline<N, T>(g.tab, ux, xl, xr, L.dir, R.dir, hinv[0], L.hinv, R.hinv, L.tau, R.tau, vnu * hinv[0], w);
    matvec_acc<N, T>(Mh, w, o);
#pragma unroll
    for (int i = 0; i < N; ++i) sw[lo + i] = o[i];
  }
  __syncthreads();
  // pass 4: y-lines: w = My w
  if (act) {
    const int i = t0, l = t1;
    T w[N], o[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      w[j] = sw[(l * N + j) * P + i];
      o[j] = T(0);
    }
    matvec_acc<N, T>(Mh, w, o);
#pragma unroll
    for (int j = 0; j < N; ++j) sw[(l * N + j) * P + i] = o[j];
  }
  __syncthreads();
  // pass 5: z-lines: dst = Mz w
  double pq = 0.0, sq = 0.0, sp = 0.0;
  if (act) {
    T w[N], o[N];
#pragma unroll
    for (int l = 0; l < N; ++l) {
      w[l] = sw[(l * N + t1) * P + t0];
      o[l] = T(0);
    }
    matvec_acc<N, T>(Mh, w, o);
    T* cd = dst + cell * N3 + t1 * N + t0;
#pragma unroll
    for (int l = 0; l < N; ++l) __builtin_nontemporal_store(o[l], cd + l * N2);
    if (partials) {
#pragma unroll
      for (int l = 0; l < N; ++l) {
        pq += static_cast<double>(u[l]) * static_cast<double>(o[l]);
        sq += static_cast<double>(o[l]);
        sp += static_cast<double>(u[l]);
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
      double x = 0, y = 0, z = 0;
      for (int k = 0; k < kApplyThreads / 64; ++k) {
        x += s_red[3 * k];
        y += s_red[3 * k + 1];
        z += s_red[3 * k + 2];
      }
      partials[4 * blockIdx.x] = x;
      partials[4 * blockIdx.x + 1] = y;
      partials[4 * blockIdx.x + 2] = z;
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
  (void)ncells;
  const int blocks = sipg_cart_blocks(N, CartGeom<double>{g.nx, g.ny, g.nz});
  if (g.allper)
    hipLaunchKernelGGL((k_sipg_cart_apply<N, T, true>), dim3(blocks), dim3(kApplyThreads), 0, s, src, dst, g, partials,
                       stop);
  else
    hipLaunchKernelGGL((k_sipg_cart_apply<N, T, false>), dim3(blocks), dim3(kApplyThreads), 0, s, src, dst, g,
                       partials, stop);
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

int sipg_cart_blocks(int n, const CartGeom<double>& g) {
  const int cpb = (kApplyThreads / (n * n)) > 0 ? kApplyThreads / (n * n) : 1;
  const int nstrip = strip_count(g.ny);
  const int hmax = g.ny / nstrip + (g.ny % nstrip ? 1 : 0);
  const int64_t per_strip = static_cast<int64_t>(g.nx) * hmax * g.nz;
  return static_cast<int>(nstrip * ((per_strip + cpb - 1) / cpb));
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
