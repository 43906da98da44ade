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
// The apply kernel uses the factored form (with V = hx hy hz)
//   H u = V (Mz x My x Mx) (mu u + sum_d (nu/h_d) Mhat^-1 A_d u)
// in five line passes (z, y, x + Mx, My, Mz) of a z-marching tile kernel
// (k_sipg_zm_apply, below); the diagonal kernel applies each A_d to unit
// vectors.
#include <atomic>

#include "internal.h"

namespace dgmf {
namespace {

// Tables and per-layer geometry are read through the constant address space:
// they are never written while a kernel runs, so uniform reads become scalar
// loads that do not wait behind the vector loads in flight.
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;

// Work decomposition of the z-marching apply: tx * ty tiles, segs z-segments
// of seglen layers; total work items spread over 8 XCDs, per_xcd each.
struct ZmPlan {
  int tx, ty, segs, seglen, total, per_xcd;
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

// Weight of the terms of boundary side f = 2d+s: 0 if it is homogeneous Neumann.
template <typename T>
__device__ __forceinline__ T bw_of(int neu, int f) {
  return ((neu >> f) & 1) ? T(0) : T(1);
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
// bwL, bwR scale a boundary face's terms: 1 on Dirichlet, 0 on homogeneous Neumann faces.
template <int N, typename T>
__device__ __forceinline__ void sipg_line(const T* __restrict__ tab, const T (&u)[N], const T (&ul)[N],
                                          const T (&ur)[N], bool dirL, bool dirR, T bwL, T bwR, T hinv, T hlinv,
                                          T hrinv, T tauL, T tauR, T sigma, T massc, T (&out)[N]) {
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
    jr = bwR * u[N - 1];
    cr = bwR * (-gu1 + T(2) * tauR * u[N - 1]);
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
    jl = bwL * u[0];
    cl = bwL * (gu0 + T(2) * tauL * u[0]);
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

// y = A x + c (c optional: accumulate into y's initial value)
template <int N, typename T>
__device__ __forceinline__ void matvec_acc(cptr<T> A, const T (&x)[N], T (&y)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T s = y[i];
#pragma unroll
    for (int j = 0; j < N; ++j) s = fma(A[i * N + j], x[j], s);
    y[i] = s;
  }
}

// w += s [ hinv (Mhat^-1 Khat u) + Mhat^-1 (face fluxes of this line) ]: one
// direction's line operator, premultiplied by the inverse 1D mass matrix.
// Face fluxes (unit tangential area): interior high face, [u] = u_N-1 - ur_0,
// {{u'}} = (l'(1).u/h + l'(0).ur/hr)/2:
//   -1/2 l'(1)_i/h [u] + delta_{i,N-1} (tau [u] - {{u'}});
// interior low face, [u] = ul_N-1 - u_0, {{u'}} = (l'(1).ul/hl + l'(0).u/h)/2:
//   -1/2 l'(0)_i/h [u] + delta_{i,0} ({{u'}} - tau [u]);
// Dirichlet faces mirror these with [u] = u and the boundary penalty 2 tau,
// scaled by bwL / bwR (0 on homogeneous Neumann faces, which add nothing).
// The low neighbour enters only through its end value ul_{N-1} and
// gl = l'(1).ul (unscaled); bline_t takes those, bline the line.
template <int N, typename T>
__device__ __forceinline__ void bline_t(cptr<T> tab, const T (&u)[N], T ul_end, T gl,
                                        const T (&ur)[N], bool dirL, bool dirR, T bwL, T bwR, T hinv, T hlinv,
                                        T hrinv, T tauL, T tauR, T s, T (&w)[N]) {
  constexpr TabLayout L{N, N};
  cptr<T> g0 = tab + L.g0();
  cptr<T> g1 = tab + L.g1();
  cptr<T> Kt = tab + L.ktil();
  cptr<T> g0t = tab + L.g0t();
  cptr<T> g1t = tab + L.g1t();
  cptr<T> e0t = tab + L.e0t();
  cptr<T> e1t = tab + L.e1t();
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
    cR = -bwR * hinv * u[N - 1];
    eR = bwR * fma(T(2) * tauR, u[N - 1], -gu1);
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
    cL = bwL * hinv * u[0];
    eL = bwL * fma(T(2) * tauL, u[0], gu0);
  } else {
    const T jump = ul_end - u[0];
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

template <int N, typename T>
__device__ __forceinline__ T dot_row(cptr<T> r, const T (&v)[N]) {
  T d = r[0] * v[0];
#pragma unroll
  for (int m = 1; m < N; ++m) d = fma(r[m], v[m], d);
  return d;
}

template <int N, typename T>
__device__ __forceinline__ void bline(cptr<T> tab, const T (&u)[N], const T (&ul)[N], const T (&ur)[N], bool dirL,
                                      bool dirR, T bwL, T bwR, T hinv, T hlinv, T hrinv, T tauL, T tauR, T s,
                                      T (&w)[N]) {
  constexpr TabLayout L{N, N};
  const T gl = dirL ? T(0) : dot_row<N, T>(tab + L.g1(), ul);
  bline_t<N, T>(tab, u, ul[N - 1], gl, ur, dirL, dirR, bwL, bwR, hinv, hlinv, hrinv, tauL, tauR, s, w);
}

// ------------------------------------------------------ z-marching apply ---
// Same factored operator and line operators as above, with a different data
// movement: a workgroup owns a TX x TY tile of cells in the x-y plane and
// marches along z over a segment of layers.  Each thread owns one z-line (i,j)
// of one tile cell; the z-lines of the layers below, at and above the current
// one stay in registers (the layer two ahead is prefetched while the current
// one is processed), so z-neighbours cost nothing extra.  x- and y-neighbour
// lines come from the tile in LDS, and only the tile rim reads neighbour cells
// from L2.  Tiles are handed to XCDs in compact bands (workgroup b runs on XCD
// b % 8), so the rim cells a workgroup reads were loaded by a tile on the same
// XCD at about the same z.
//
// Tile per degree and element size (bytes).  Where n^2 divides 64 or one cell
// nearly fills a wavefront, a cell's n^2 threads stay inside one wavefront
// and the transposes of its own lines need only wavefront ordering.  Where
// that would idle many lanes (n = 5: 50 of 64, n = 6: 36, n = 7: 49), PACK
// numbers the threads of the tile's cells consecutively across wavefronts,
// so a cell may straddle two of them and those transposes take workgroup
// barriers.
template <int N, int ES>
struct ZmTile {
  static constexpr int TX = 2, TY = 2;
  static constexpr bool PACK = false;
};
template <int ES> struct ZmTile<2, ES> { static constexpr int TX = 8, TY = 8; static constexpr bool PACK = false; };
template <int ES> struct ZmTile<3, ES> { static constexpr int TX = 4, TY = 7; static constexpr bool PACK = false; };
template <> struct ZmTile<4, 8> { static constexpr int TX = 4, TY = 4; static constexpr bool PACK = false; };
template <> struct ZmTile<4, 4> { static constexpr int TX = 8, TY = 4; static constexpr bool PACK = false; };
template <int ES> struct ZmTile<5, ES> { static constexpr int TX = 5, TY = 2; static constexpr bool PACK = true; };
template <> struct ZmTile<6, 8> { static constexpr int TX = 7, TY = 2; static constexpr bool PACK = true; };
template <> struct ZmTile<6, 4> { static constexpr int TX = 3, TY = 2; static constexpr bool PACK = true; };
template <> struct ZmTile<7, 8> { static constexpr int TX = 5, TY = 1; static constexpr bool PACK = true; };
template <> struct ZmTile<8, 8> { static constexpr int TX = 4, TY = 2; static constexpr bool PACK = false; };

template <int N, typename T>
struct Zm {
  using Tile = ZmTile<N, int(sizeof(T))>;
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int P = (N % 2) ? N : N + 1;
  static constexpr int CL = N2 * P;
  static constexpr int TX = Tile::TX, TY = Tile::TY, NC = TX * TY;
  static constexpr bool PACK = Tile::PACK;
  static constexpr int CPW = 64 / N2;                       // whole cells per wavefront
  static constexpr int THREADS = PACK ? ((NC * N2 + 63) / 64) * 64 : ((NC + CPW - 1) / CPW) * 64;
};


// Orders this wavefront's LDS accesses (all lanes of a cell are in it).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Orders the LDS accesses of every thread of a cell: the wavefront when a
// cell never leaves it, else the workgroup.
template <bool PACK>
__device__ __forceinline__ void cell_sync() {
  if constexpr (PACK) __syncthreads();
  else wave_sync();
}

// The z-line (i, j) = off of a cell: n values, stride n^2 (coalesced across the
// n^2 threads of a cell).
template <int N, typename T>
__device__ __forceinline__ void load_zline(const T* __restrict__ src, int cell, int off, T (&v)[N]) {
  constexpr int N2 = N * N, N3 = N2 * N;
#pragma unroll
  for (int l = 0; l < N; ++l) v[l] = src[cell * N3 + off + l * N2];
}

// Line operator of direction d on a uniform, fully periodic mesh (tables
// UTab, pre-scaled on the host): w += A_d u + ur_0 G1_d + bR E1 + ul_{n-1} G0_d
// + bL E0 with bR = c_d (u_{n-1} - ur_0) + g0s_d.ur, bL = c_d (u_0 - ul_{n-1}) + g1s_d.ul.
// (uline_t: the low neighbour given by ul_{n-1} and dl = g1s_d.ul)
template <int N, typename T>
__device__ __forceinline__ void uline_t(cptr<T> ut, int d, const T (&u)[N], T ul_end, T dl, const T (&ur)[N],
                                        T (&w)[N]) {
  constexpr UTab L{N};
  const cptr<T> A = ut + L.A(d), G1 = ut + L.G1(d), G0 = ut + L.G0(d), g0s = ut + L.g0s(d);
  const cptr<T> E1 = ut + L.E1(), E0 = ut + L.E0();
  const T c = ut[L.c(d)];
  T dr = g0s[0] * ur[0];
#pragma unroll
  for (int m = 1; m < N; ++m) dr = fma(g0s[m], ur[m], dr);
  const T bR = fma(c, u[N - 1] - ur[0], dr);
  const T bL = fma(c, u[0] - ul_end, dl);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    T acc = fma(G1[i], ur[0], fma(E1[i], bR, fma(G0[i], ul_end, fma(E0[i], bL, w[i]))));
#pragma unroll
    for (int m = 0; m < N; ++m) acc = fma(A[i * N + m], u[m], acc);
    w[i] = acc;
  }
}

template <int N, typename T>
__device__ __forceinline__ void uline(cptr<T> ut, int d, const T (&u)[N], const T (&ul)[N], const T (&ur)[N],
                                      T (&w)[N]) {
  constexpr UTab L{N};
  uline_t<N, T>(ut, d, u, ul[N - 1], dot_row<N, T>(ut + L.g1s(d), ul), ur, w);
}

// Work state of one workgroup of the z-marching apply.
template <int N, typename T>
struct ZmCtx {
  static constexpr int N2 = N * N, N3 = N2 * N, P = Zm<N, T>::P, CL = Zm<N, T>::CL;
  static constexpr int NR = 2 * (Zm<N, T>::TX + Zm<N, T>::TY);                    // rim cells per layer
  static constexpr int RPT = (NR * N3 + Zm<N, T>::THREADS - 1) / Zm<N, T>::THREADS;  // rim values per thread
  bool act, zper;
  int col, nxy, zoff, slot, t0, t1;
  T hx, hy, hinvx, hinvy, tpx, tpy;
  bool xl_dir, xr_dir, yl_dir, yr_dir;
  T xl_hinv, xr_hinv, yl_hinv, yr_hinv, xl_tp, xr_tp, yl_tp, yr_tp;
  int xl_nb, xr_nb, yl_nb, yr_nb;   // LDS offset of the neighbour cell (tile slot or rim slot)
  T rim[RPT];                       // rim values of the next layer, in flight
};

// One layer of the march.  W: z-line window (layer offset -1, 0, +1, and the
// slot that receives layer +2).
template <int N, typename T, bool PER, bool UNI, bool EPI>
__device__ __forceinline__ void zm_layer(const T* __restrict__ src, T* __restrict__ dst, const CartGeom<T>& g,
                                         ZmCtx<N, T>& c, int cz, int z1, T* s_u, T* s_w, T* s_rim_next,
                                         const int* s_rimcol, cptr<T> tab, cptr<T> gh, cptr<T> ghinv,
                                         cptr<T> gtp, T& up_end, T& up_dot, const T (&uc)[N], const T (&un)[N],
                                         T (&unn)[N], bool want_partials, double& pq, double& sq, double& sp,
                                         const ChebEpi<T>& epi) {
  using C = ZmCtx<N, T>;
  constexpr int N2 = C::N2, N3 = C::N3, P = C::P, NR = C::NR, RPT = C::RPT, TH = Zm<N, T>::THREADS;
  const int tid = threadIdx.x;
  const int t0 = c.t0, t1 = c.t1;
  T* su = s_u + c.slot;
  T* sw = s_w + c.slot;
  wave_sync();   // the previous layer's last reads of sw by this wavefront
  // prefetch: z-lines two layers ahead (own column), rim cells one layer ahead (whole workgroup)
  if (cz + 1 < z1) {
    const int zq = cz + 2;
    if (c.act && (zq < g.nz || c.zper)) load_zline<N, T>(src, (zq >= g.nz ? zq - g.nz : zq) * c.nxy + c.col, c.zoff, unn);
    const int lay1 = (cz + 1) * c.nxy;
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int e = tid + k * TH;
      if (e < NR * N3) {
        const int r = e / N3;
        const int rc = s_rimcol[r];
        if (rc >= 0) c.rim[k] = src[(lay1 + rc) * N3 + (e - r * N3)];
      }
    }
  }
  const cptr<T> ut = (cptr<T>)(g.utab);
  // layer geometry (uniform: scalar loads)
  const T hz = UNI ? T(0) : gh[cz], hinvz = UNI ? T(0) : ghinv[cz], tpz = UNI ? T(0) : gtp[cz];
  int zlo = cz - 1, zhi = cz + 1;
  const bool zl_dir = zlo < 0 && !c.zper, zr_dir = zhi >= g.nz && !c.zper;
  zlo = zlo < 0 ? g.nz - 1 : zlo;
  zhi = zhi >= g.nz ? 0 : zhi;
  const T zl_hinv = (UNI || zl_dir) ? T(0) : ghinv[zlo], zr_hinv = (UNI || zr_dir) ? T(0) : ghinv[zhi];
  const T zl_tp = UNI ? T(0) : gtp[zlo], zr_tp = UNI ? T(0) : gtp[zhi];
  const T tau_c = g.pen * (c.tpx + c.tpy + tpz);
  const T vol = c.hx * c.hy * hz;
  const T vnu = vol * g.nu;
  // pass 1: z-lines from registers: w = mu V u + B_z u
  if (c.act) {
    T w[N];
    if constexpr (UNI) {
#pragma unroll
      for (int l = 0; l < N; ++l) w[l] = T(0);
      uline_t<N, T>(ut, 2, uc, up_end, up_dot, un, w);
    } else {
      const T tzl = zl_dir ? tau_c : fmax(tau_c, g.pen * (c.tpx + c.tpy + zl_tp));
      const T tzr = zr_dir ? tau_c : fmax(tau_c, g.pen * (c.tpx + c.tpy + zr_tp));
      const T mv = g.mu * vol;
#pragma unroll
      for (int l = 0; l < N; ++l) w[l] = mv * uc[l];
      bline_t<N, T>(tab, uc, up_end, up_dot, un, zl_dir, zr_dir, bw_of<T>(g.neu, 4), bw_of<T>(g.neu, 5), hinvz,
                    zl_hinv, zr_hinv, tzl, tzr, vnu * hinvz, w);
    }
#pragma unroll
    for (int l = 0; l < N; ++l) {
      su[(l * N + t1) * P + t0] = uc[l];
      sw[(l * N + t1) * P + t0] = w[l];
    }
  }
  // this layer's high-face trace is the next layer's low-neighbour trace
  up_end = uc[N - 1];
  if constexpr (UNI) up_dot = dot_row<N, T>(ut + UTab{N}.g1s(2), uc);
  else up_dot = dot_row<N, T>(tab + TabLayout{N, N}.g1(), uc);
  __syncthreads();
  // pass 2: y-lines (i, l) = (t0, t1): w += B_y u
  if (c.act) {
    const int i = t0, l = t1;
    const T* nl = s_u + c.yl_nb;
    const T* nr = s_u + c.yr_nb;
    T uy[N], vl[N], vr[N], w[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const int e = (l * N + j) * P + i;
      uy[j] = su[e];
      w[j] = sw[e];
      vl[j] = nl[e];
      vr[j] = nr[e];
    }
    if constexpr (UNI) {
      uline<N, T>(ut, 1, uy, vl, vr, w);
    } else {
      const T tl = c.yl_dir ? tau_c : fmax(tau_c, g.pen * (c.tpx + c.yl_tp + tpz));
      const T tr = c.yr_dir ? tau_c : fmax(tau_c, g.pen * (c.tpx + c.yr_tp + tpz));
      bline<N, T>(tab, uy, vl, vr, c.yl_dir, c.yr_dir, bw_of<T>(g.neu, 2), bw_of<T>(g.neu, 3), c.hinvy, c.yl_hinv,
                  c.yr_hinv, tl, tr, vnu * c.hinvy, w);
    }
#pragma unroll
    for (int j = 0; j < N; ++j) sw[(l * N + j) * P + i] = w[j];
  }
  cell_sync<Zm<N, T>::PACK>();
  // pass 3: x-lines (j, l) = (t0, t1): w += B_x u, then w = Mx w
  if (c.act) {
    const int lo = (t1 * N + t0) * P;
    const T* nl = s_u + c.xl_nb;
    const T* nr = s_u + c.xr_nb;
    T ux[N], vl[N], vr[N], w[N], o[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      ux[i] = su[lo + i];
      w[i] = sw[lo + i];
      vl[i] = nl[lo + i];
      vr[i] = nr[lo + i];
      o[i] = T(0);
    }
    if constexpr (UNI) {
      uline<N, T>(ut, 0, ux, vl, vr, w);
    } else {
      const T tl = c.xl_dir ? tau_c : fmax(tau_c, g.pen * (c.xl_tp + c.tpy + tpz));
      const T tr = c.xr_dir ? tau_c : fmax(tau_c, g.pen * (c.xr_tp + c.tpy + tpz));
      bline<N, T>(tab, ux, vl, vr, c.xl_dir, c.xr_dir, bw_of<T>(g.neu, 0), bw_of<T>(g.neu, 1), c.hinvx, c.xl_hinv,
                  c.xr_hinv, tl, tr, vnu * c.hinvx, w);
    }
    matvec_acc<N, T>(tab, w, o);
#pragma unroll
    for (int i = 0; i < N; ++i) sw[lo + i] = o[i];
  }
  __syncthreads();   // every wavefront is done with s_u (tile and rim) of this layer
  // pass 4: y-lines: w = My w
  if (c.act) {
    const int i = t0, l = t1;
    T w[N], o[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      w[j] = sw[(l * N + j) * P + i];
      o[j] = T(0);
    }
    matvec_acc<N, T>(tab, w, o);
#pragma unroll
    for (int j = 0; j < N; ++j) sw[(l * N + j) * P + i] = o[j];
  }
  cell_sync<Zm<N, T>::PACK>();
  // pass 5: z-lines: dst = Mz w (coalesced store); the rim of the next layer goes to LDS
  if (c.act) {
    T w[N], o[N];
    const int at = (cz * c.nxy + c.col) * N3 + c.zoff;
    T* cd = dst + at;
    T eb[N], ed[N], ep[N];
    if constexpr (EPI) {   // issued before the sweep so that their latency overlaps it
#pragma unroll
      for (int l = 0; l < N; ++l) {
        eb[l] = epi.b[at + l * N2];
        ed[l] = epi.dinv[at + l * N2];
        ep[l] = epi.prev_zero ? T(0) : cd[l * N2];
      }
    }
#pragma unroll
    for (int l = 0; l < N; ++l) {
      w[l] = sw[(l * N + t1) * P + t0];
      o[l] = T(0);
    }
    matvec_acc<N, T>(tab, w, o);
    if constexpr (EPI) {
#pragma unroll
      for (int l = 0; l < N; ++l)
        o[l] = fma(epi.c2 * ed[l], eb[l] - o[l], fma(epi.c1, uc[l] - ep[l], uc[l]));
    }
#pragma unroll
    for (int l = 0; l < N; ++l) __builtin_nontemporal_store(o[l], cd + l * N2);
    if (want_partials) {
#pragma unroll
      for (int l = 0; l < N; ++l) {
        pq += static_cast<double>(uc[l]) * static_cast<double>(o[l]);
        sq += static_cast<double>(o[l]);
        sp += static_cast<double>(uc[l]);
      }
    }
  }
  if (cz + 1 < z1) {
#pragma unroll
    for (int k = 0; k < RPT; ++k) {
      const int e = tid + k * TH;
      if (e < NR * N3) {
        const int r = e / N3, q = e - r * N3;
        s_rim_next[r * C::CL + (q / N) * P + q % N] = c.rim[k];
      }
    }
  }
}

template <int N, typename T, bool PER, bool UNI, bool EPI>
__global__ void __launch_bounds__((Zm<N, T>::THREADS)) k_sipg_zm_apply(const T* __restrict__ src, T* __restrict__ dst,
                                                                 const CartGeom<T> g, const ZmPlan pl,
                                                                 double* __restrict__ partials, const int* stop,
                                                                 const ChebEpi<T> epi) {
  if (stop && *stop) return;   // uniform for the whole grid: CG already finished
  using Z = Zm<N, T>;
  using C = ZmCtx<N, T>;
  constexpr int N3 = Z::N3, P = Z::P, CL = Z::CL, TX = Z::TX, TY = Z::TY, NC = Z::NC, NR = C::NR;
  // s_u holds the tile cells followed by the rim cells: neighbour lines are
  // read from one array whether the neighbour is in the tile or not.
  // s_u holds the tile cells followed by the rim cells, so neighbour lines are
  // read from one array whether the neighbour is in the tile or not; s_w is
  // private to each cell's wavefront.
  __shared__ T s_u[1][(NC + NR) * CL];
  __shared__ T s_w[NC * CL];
  __shared__ int s_rimcol[NR];
  __shared__ double s_red[3 * (Z::THREADS / 64)];
  const cptr<T> tab = (cptr<T>)(g.tab);
  const cptr<T> gh = (cptr<T>)(g.h[2]);
  const cptr<T> ghinv = (cptr<T>)(g.hinv[2]);
  const cptr<T> gtp = (cptr<T>)(g.tp[2]);
  const int tid = threadIdx.x;
  const int item = (blockIdx.x % 8) * pl.per_xcd + blockIdx.x / 8;
  double pq = 0.0, sq = 0.0, sp = 0.0;
  if (item < pl.total) {   // uniform over the workgroup
    const int ntile = pl.tx * pl.ty;
    const int seg = item / ntile, tile = item - seg * ntile;
    const int tyi = tile / pl.tx, txi = tile - tyi * pl.tx;
    const int x0 = txi * TX, y0 = tyi * TY;
    const int wx = g.nx - x0 < TX ? g.nx - x0 : TX;   // active tile extent
    const int wy = g.ny - y0 < TY ? g.ny - y0 : TY;
    const int z0 = seg * pl.seglen;
    const int z1 = z0 + pl.seglen < g.nz ? z0 + pl.seglen : g.nz;
    C c;
    int lc, t;   // tile cell (NC: none) and thread within the cell
    if constexpr (Z::PACK) {
      lc = tid / Z::N2;
      t = tid - lc * Z::N2;
      lc = lc < NC ? lc : NC;
    } else {
      const int lane = tid & 63, cw = lane / Z::N2;
      lc = cw < Z::CPW ? (tid >> 6) * Z::CPW + cw : NC;
      t = lane - cw * Z::N2;
    }
    c.t0 = t % N;
    c.t1 = t / N;
    const int a = lc % TX, b = lc / TX;
    const int cx = x0 + a, cy = y0 + b;
    c.act = lc < NC && a < wx && b < wy;
    c.slot = (lc < NC ? lc : 0) * CL;
    c.nxy = g.nx * g.ny;
    c.col = c.act ? cy * g.nx + cx : 0;
    c.zoff = c.t1 * N + c.t0;
    c.zper = PER || g.per[2];
    // rim cells: [0,TX) y-low of column a, [TX,2TX) y-high, then x-low / x-high of row b
    if (tid < NR) {
      int r = tid, col = -1;
      if (r < 2 * TX) {
        const int aa = r % TX, hi = r / TX;
        if (aa < wx) {
          int yy = hi ? y0 + wy : y0 - 1;
          if (yy < 0 || yy >= g.ny) yy = (PER || g.per[1]) ? (yy < 0 ? g.ny - 1 : 0) : -1;
          const bool inside = yy >= y0 && yy < y0 + wy;
          if (yy >= 0 && !inside) col = yy * g.nx + x0 + aa;
        }
      } else {
        r -= 2 * TX;
        const int bb = r % TY, hi = r / TY;
        if (bb < wy) {
          int xx = hi ? x0 + wx : x0 - 1;
          if (xx < 0 || xx >= g.nx) xx = (PER || g.per[0]) ? (xx < 0 ? g.nx - 1 : 0) : -1;
          const bool inside = xx >= x0 && xx < x0 + wx;
          if (xx >= 0 && !inside) col = (y0 + bb) * g.nx + xx;
        }
      }
      s_rimcol[tid] = col;
    }
    // per-column geometry and neighbour slots (x and y do not change along the march)
    c.hx = c.hy = c.hinvx = c.hinvy = c.tpx = c.tpy = T(0);
    c.xl_dir = c.xr_dir = c.yl_dir = c.yr_dir = true;
    c.xl_hinv = c.xr_hinv = c.yl_hinv = c.yr_hinv = c.xl_tp = c.xr_tp = c.yl_tp = c.yr_tp = T(0);
    c.xl_nb = c.xr_nb = c.yl_nb = c.yr_nb = c.slot;
#pragma unroll
    for (int k = 0; k < C::RPT; ++k) c.rim[k] = T(0);
    if (c.act) {
      c.hx = g.h[0][cx];
      c.hy = g.h[1][cy];
      c.hinvx = g.hinv[0][cx];
      c.hinvy = g.hinv[1][cy];
      c.tpx = g.tp[0][cx];
      c.tpy = g.tp[1][cy];
      // x-low
      int n = cx - 1;
      if (n < 0) n = (PER || g.per[0]) ? g.nx - 1 : -1;
      if (n >= 0) {
        c.xl_dir = false;
        c.xl_hinv = g.hinv[0][n];
        c.xl_tp = g.tp[0][n];
        c.xl_nb = (n >= x0 && n < x0 + wx) ? (lc + (n - cx)) * CL : (NC + 2 * TX + b) * CL;
      }
      n = cx + 1;
      if (n >= g.nx) n = (PER || g.per[0]) ? 0 : -1;
      if (n >= 0) {
        c.xr_dir = false;
        c.xr_hinv = g.hinv[0][n];
        c.xr_tp = g.tp[0][n];
        c.xr_nb = (n >= x0 && n < x0 + wx) ? (lc + (n - cx)) * CL : (NC + 2 * TX + TY + b) * CL;
      }
      n = cy - 1;
      if (n < 0) n = (PER || g.per[1]) ? g.ny - 1 : -1;
      if (n >= 0) {
        c.yl_dir = false;
        c.yl_hinv = g.hinv[1][n];
        c.yl_tp = g.tp[1][n];
        c.yl_nb = (n >= y0 && n < y0 + wy) ? (lc + (n - cy) * TX) * CL : (NC + a) * CL;
      }
      n = cy + 1;
      if (n >= g.ny) n = (PER || g.per[1]) ? 0 : -1;
      if (n >= 0) {
        c.yr_dir = false;
        c.yr_hinv = g.hinv[1][n];
        c.yr_tp = g.tp[1][n];
        c.yr_nb = (n >= y0 && n < y0 + wy) ? (lc + (n - cy) * TX) * CL : (NC + TX + a) * CL;
      }
    }
    // z-line window: slots hold layers z0 and z0+1 (slot 2 receives z0+2);
    // the layer below enters only through its high-face trace (end value and
    // end derivative)
    T z[3][N];
#pragma unroll
    for (int s = 0; s < 3; ++s)
#pragma unroll
      for (int l = 0; l < N; ++l) z[s][l] = T(0);
    T up_end = T(0), up_dot = T(0);
    if (c.act) {
      const int zl = z0 - 1, zr = z0 + 1;
      if (zl >= 0 || c.zper) {
        load_zline<N, T>(src, (zl < 0 ? g.nz - 1 : zl) * c.nxy + c.col, c.zoff, z[2]);
        up_end = z[2][N - 1];
        if constexpr (UNI) up_dot = dot_row<N, T>((cptr<T>)(g.utab) + UTab{N}.g1s(2), z[2]);
        else up_dot = dot_row<N, T>(tab + TabLayout{N, N}.g1(), z[2]);
      }
      load_zline<N, T>(src, z0 * c.nxy + c.col, c.zoff, z[0]);
      if (zr < g.nz || c.zper) load_zline<N, T>(src, (zr >= g.nz ? 0 : zr) * c.nxy + c.col, c.zoff, z[1]);
    }
    __syncthreads();   // s_rimcol
    // rim of the first layer
#pragma unroll
    for (int k = 0; k < C::RPT; ++k) {
      const int e = tid + k * Z::THREADS;
      if (e < NR * N3) {
        const int r = e / N3, q = e - r * N3;
        const int rc = s_rimcol[r];
        if (rc >= 0) s_u[0][(NC + r) * CL + (q / N) * P + q % N] = src[(z0 * c.nxy + rc) * N3 + q];
      }
    }
    // s_rim is read after the first barrier inside zm_layer
    const bool wp = partials != nullptr;
    T* const su = s_u[0];
#pragma unroll 1
    for (int cz = z0; cz < z1; cz += 3) {
      zm_layer<N, T, PER, UNI, EPI>(src, dst, g, c, cz, z1, su, s_w, su + NC * CL, s_rimcol, tab, gh, ghinv, gtp,
                                    up_end, up_dot, z[0], z[1], z[2], wp, pq, sq, sp, epi);
      if (cz + 1 < z1)
        zm_layer<N, T, PER, UNI, EPI>(src, dst, g, c, cz + 1, z1, su, s_w, su + NC * CL, s_rimcol, tab, gh, ghinv,
                                      gtp, up_end, up_dot, z[1], z[2], z[0], wp, pq, sq, sp, epi);
      if (cz + 2 < z1)
        zm_layer<N, T, PER, UNI, EPI>(src, dst, g, c, cz + 2, z1, su, s_w, su + NC * CL, s_rimcol, tab, gh, ghinv,
                                      gtp, up_end, up_dot, z[2], z[0], z[1], wp, pq, sq, sp, epi);
    }
  }
  if (partials) {
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
      double x = 0, y = 0, zz = 0;
      for (int k = 0; k < Zm<N, T>::THREADS / 64; ++k) {
        x += s_red[3 * k];
        y += s_red[3 * k + 1];
        zz += s_red[3 * k + 2];
      }
      partials[4 * blockIdx.x] = x;
      partials[4 * blockIdx.x + 1] = y;
      partials[4 * blockIdx.x + 2] = zz;
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
    sipg_line<N, T>(g.tab, e, el, er, !hasL, !hasR, bw_of<T>(g.neu, 2 * d), bw_of<T>(g.neu, 2 * d + 1), ci.hinv[d],
                    hl, hr, tauL, tauR, sigma, massc, out);
    T v = out[0];
#pragma unroll
    for (int m = 1; m < N; ++m) v = (m == p) ? out[m] : v;
    dd[d] = v;
  }
  diag[gid] = dd[0] * md[1] * md[2] + md[0] * dd[1] * md[2] + md[0] * md[1] * dd[2];
}

// Workgroups of `kernel` (`threads` each) resident on the current device at
// once, by the runtime's occupancy calculator (registers, LDS, wavefronts).
int resident_blocks(const void* kernel, int threads) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) cus = 1;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kernel, threads, 0) != hipSuccess || per < 1) per = 1;
  return per * cus;
}

// resident_blocks of one apply kernel, kept per device after the first query
template <int N, typename T, bool PER, bool UNI, bool EPI>
int zm_resident() {
  static std::atomic<int> cache[16];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  const void* k = reinterpret_cast<const void*>(&k_sipg_zm_apply<N, T, PER, UNI, EPI>);
  if (dev < 0 || dev >= 16) return resident_blocks(k, Zm<N, T>::THREADS);
  int r = cache[dev].load(std::memory_order_relaxed);
  if (r == 0) {
    r = resident_blocks(k, Zm<N, T>::THREADS);
    cache[dev].store(r, std::memory_order_relaxed);
  }
  return r;
}

// z-segments of the march: a workgroup per (tile, segment), `resident` of them
// running at once.  The segment count minimises rounds x (layers per segment
// + 2), the 2 standing for the set-up of a segment (its first two z-lines);
// a mesh whose every layer fits one round (coarse multigrid levels) may go
// down to one layer per workgroup, a larger one to kMinLayers.
template <int N, typename T>
ZmPlan zm_plan_n(int nx, int ny, int nz, int resident) {
  constexpr int TX = Zm<N, T>::TX, TY = Zm<N, T>::TY;
  constexpr int kMinLayers = 4;
  ZmPlan p{};
  p.tx = (nx + TX - 1) / TX;
  p.ty = (ny + TY - 1) / TY;
  const int64_t tiles = static_cast<int64_t>(p.tx) * p.ty;
  const int minl = tiles * nz <= resident ? 1 : kMinLayers;
  const int maxseg = nz / minl > 1 ? nz / minl : 1;
  int64_t best = -1;
  p.seglen = nz;
  for (int segs = 1; segs <= maxseg; ++segs) {
    const int len = (nz + segs - 1) / segs;
    const int64_t sg = (nz + len - 1) / len;
    const int64_t cost = ((tiles * sg + resident - 1) / resident) * (len + 2);
    if (best < 0 || cost < best) {
      best = cost;
      p.seglen = len;
    }
  }
  p.segs = (nz + p.seglen - 1) / p.seglen;
  p.total = static_cast<int>(tiles * p.segs);
  p.per_xcd = (p.total + 7) / 8;
  return p;
}

// plan and grid of the apply variant that geometry g selects
template <int N, typename T, bool EPI>
ZmPlan zm_plan_for(const CartGeom<T>& g) {
  const int r = g.utab ? zm_resident<N, T, true, true, EPI>()
                       : (g.allper ? zm_resident<N, T, true, false, EPI>() : zm_resident<N, T, false, false, EPI>());
  return zm_plan_n<N, T>(g.nx, g.ny, g.nz, r);
}

ZmPlan zm_plan(int n, const CartGeom<double>& g) {
  switch (n) {
    case 2: return zm_plan_for<2, double, false>(g);
    case 3: return zm_plan_for<3, double, false>(g);
    case 4: return zm_plan_for<4, double, false>(g);
    case 5: return zm_plan_for<5, double, false>(g);
    case 6: return zm_plan_for<6, double, false>(g);
    case 7: return zm_plan_for<7, double, false>(g);
    default: return zm_plan_for<8, double, false>(g);
  }
}

template <int N, typename T, bool EPI>
dgmf_status launch_apply_n(const CartGeom<T>& g, const T* src, T* dst, int64_t ncells, double* partials,
                           const int* stop, const ChebEpi<T>& epi, hipStream_t s) {
  (void)ncells;
  // partial sums come with the fp64 apply only: one row per workgroup of the
  // fp64 plan, the count sipg_cart_blocks reports
  if (partials && sizeof(T) != 8) return fail(DGMF_UNSUPPORTED, "k_sipg_zm_apply: partial sums need fp64");
  const ZmPlan pl = zm_plan_for<N, T, EPI>(g);
  const int blocks = 8 * pl.per_xcd;
  if (g.utab)
    hipLaunchKernelGGL((k_sipg_zm_apply<N, T, true, true, EPI>), dim3(blocks), dim3(Zm<N, T>::THREADS), 0, s, src, dst,
                       g, pl, partials, stop, epi);
  else if (g.allper)
    hipLaunchKernelGGL((k_sipg_zm_apply<N, T, true, false, EPI>), dim3(blocks), dim3(Zm<N, T>::THREADS), 0, s, src,
                       dst, g, pl, partials, stop, epi);
  else
    hipLaunchKernelGGL((k_sipg_zm_apply<N, T, false, false, EPI>), dim3(blocks), dim3(Zm<N, T>::THREADS), 0, s, src,
                       dst, g, pl, partials, stop, epi);
  DGMF_LAUNCH_CHECK("k_sipg_zm_apply");
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

int sipg_cart_blocks(int n, const CartGeom<double>& g) { return 8 * zm_plan(n, g).per_xcd; }

namespace {
template <int N>
void prime_n() {
  (void)zm_resident<N, double, true, true, false>();
  (void)zm_resident<N, double, true, false, false>();
  (void)zm_resident<N, double, false, false, false>();
  (void)zm_resident<N, double, true, true, true>();
  (void)zm_resident<N, double, true, false, true>();
  (void)zm_resident<N, double, false, false, true>();
  (void)zm_resident<N, float, true, true, false>();
  (void)zm_resident<N, float, true, false, false>();
  (void)zm_resident<N, float, false, false, false>();
  (void)zm_resident<N, float, true, true, true>();
  (void)zm_resident<N, float, true, false, true>();
  (void)zm_resident<N, float, false, false, true>();
}
}  // namespace

void sipg_cart_prime(int n) {
  switch (n) {
    case 2: prime_n<2>(); break;
    case 3: prime_n<3>(); break;
    case 4: prime_n<4>(); break;
    case 5: prime_n<5>(); break;
    case 6: prime_n<6>(); break;
    case 7: prime_n<7>(); break;
    case 8: prime_n<8>(); break;
    default: break;
  }
}

template <typename T>
dgmf_status launch_sipg_cart_apply(int n, const CartGeom<T>& g, const T* src, T* dst, int64_t ncells,
                                   double* partials, const int* stop, hipStream_t s) {
  const ChebEpi<T> none{nullptr, nullptr, T(0), T(0), 1};
  switch (n) {
    case 2: return launch_apply_n<2, T, false>(g, src, dst, ncells, partials, stop, none, s);
    case 3: return launch_apply_n<3, T, false>(g, src, dst, ncells, partials, stop, none, s);
    case 4: return launch_apply_n<4, T, false>(g, src, dst, ncells, partials, stop, none, s);
    case 5: return launch_apply_n<5, T, false>(g, src, dst, ncells, partials, stop, none, s);
    case 6: return launch_apply_n<6, T, false>(g, src, dst, ncells, partials, stop, none, s);
    case 7: return launch_apply_n<7, T, false>(g, src, dst, ncells, partials, stop, none, s);
    case 8: return launch_apply_n<8, T, false>(g, src, dst, ncells, partials, stop, none, s);
    default: return fail(DGMF_UNSUPPORTED, "degree %d not built", n - 1);
  }
}

template <typename T>
dgmf_status launch_sipg_cart_cheb(int n, const CartGeom<T>& g, const T* xk, T* dst, const ChebEpi<T>& epi,
                                  const int* stop, hipStream_t s) {
  const int64_t nc = static_cast<int64_t>(g.nx) * g.ny * g.nz;
  switch (n) {
    case 2: return launch_apply_n<2, T, true>(g, xk, dst, nc, nullptr, stop, epi, s);
    case 3: return launch_apply_n<3, T, true>(g, xk, dst, nc, nullptr, stop, epi, s);
    case 4: return launch_apply_n<4, T, true>(g, xk, dst, nc, nullptr, stop, epi, s);
    case 5: return launch_apply_n<5, T, true>(g, xk, dst, nc, nullptr, stop, epi, s);
    case 6: return launch_apply_n<6, T, true>(g, xk, dst, nc, nullptr, stop, epi, s);
    case 7: return launch_apply_n<7, T, true>(g, xk, dst, nc, nullptr, stop, epi, s);
    case 8: return launch_apply_n<8, T, true>(g, xk, dst, nc, nullptr, stop, epi, s);
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
template dgmf_status launch_sipg_cart_cheb<double>(int, const CartGeom<double>&, const double*, double*,
                                                   const ChebEpi<double>&, const int*, hipStream_t);
template dgmf_status launch_sipg_cart_cheb<float>(int, const CartGeom<float>&, const float*, float*,
                                                  const ChebEpi<float>&, const int*, hipStream_t);
template dgmf_status launch_sipg_cart_diag<double>(int, const CartGeom<double>&, double*, int64_t, hipStream_t);
template dgmf_status launch_sipg_cart_diag<float>(int, const CartGeom<float>&, float*, int64_t, hipStream_t);

}  // namespace dgmf
