// SIPG Laplace / Helmholtz apply with geometry stored at every quadrature
// point (gfx950): the sum-factorised evaluation of Sec. 5 for general
// (parallelepiped) affine cells, streaming the metric from HBM.
//
// Stored geometry (filled once per mesh by k_metric_fill):
//   cell point q:  G = w_q detJ J^{-1} J^{-T} (6 symmetric entries), m = w_q detJ
//   face point q:  wdA = tangential weight x surface Jacobian,
//                  vL = J_L^{-1} n wdA, vR = J_R^{-1} n wdA   (n: unit normal from L to R;
//                  on a boundary face L is the cell and n points outwards)
//   face:          tau geometry (k+1)^2 (A_int/2 + A_Dir)/V, maximum over both cells.
// With hat-gradients of the reference basis,
//   (grad v, grad u)_K = sum_q hat(grad v)^T G hat(grad u),
//   (grad u . n) wdA   = hat(grad u) . (J^{-1} n wdA).
// Interior faces (Sec. 3.2, eqs. ipflux, tau), [u] = uL - uR, {{du/dn}} over both sides:
//   - ({{grad v}}.n, [u]) - ([v], {{grad u}}.n) + tau ([v], [u])
// Dirichlet faces: - (grad v.n, u) - (v, grad u.n) + 2 tau (v, u); homogeneous
// Neumann faces: nothing (Sec. 3.2: own-trace flux, gradient flux is data).
//
// Kernel layout: the n^2 lanes of a cell sit in one wavefront (several cells
// per wavefront when n^2 <= 32, four wavefronts per workgroup); the cell's
// point fields live in LDS and the sweeps go line by line over its lanes.
// Own face traces are extrapolated from the Gauss-point data along the normal
// lines and the face terms are injected back into the point fluxes, so the
// transposed cell sweeps lift cell and face terms together.  A neighbour's
// traces come through LDS from the neighbouring cell itself when both sit in
// one 2x2x2 block of the workgroup (degrees 1, 3, 4), else from the
// neighbour's nodal face planes.  An optional epilogue fuses the Chebyshev
// step of the smoother and preconditioner into the store.
#include "curv_map.h"
#include "internal.h"

namespace dgmf {
namespace {


// ----------------------------------------------------------- table layout
struct MTab {
  int n;
  __host__ __device__ int S() const { return 0; }
  __host__ __device__ int D() const { return n * n; }
  __host__ __device__ int Dg() const { return 2 * n * n; }
  __host__ __device__ int g0() const { return 3 * n * n; }
  __host__ __device__ int g1() const { return 3 * n * n + n; }
  __host__ __device__ int w() const { return 3 * n * n + 2 * n; }
  // Lagrange basis on the Gauss points evaluated at 0 and 1: the value at a
  // face of any polynomial of degree < n along the normal line
  __host__ __device__ int e0() const { return 3 * n * n + 3 * n; }
  __host__ __device__ int e1() const { return 3 * n * n + 4 * n; }
  __host__ __device__ int size() const { return 3 * n * n + 5 * n; }
};

// ------------------------------------------------------------ LDS sweeps
// Work of one cell is done by the n^2 lanes of that cell, which all sit in
// one wavefront (several cells per wavefront when n^2 <= 32): the LDS
// exchanges between the steps below only need this wavefront's ordering.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// load through a global-memory pointer (the face metric pointers are chosen
// among several arrays, which hides their address space from the compiler)
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
  return *(const __attribute__((address_space(1))) T*)p;
}

template <int N>
struct MetShape {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int CPW = 64 / N2;              // cells per wavefront
  static constexpr int WAVES = 4;
  static constexpr int CPB = CPW * WAVES;          // cells per workgroup
  static constexpr int THREADS = 64 * WAVES;
  // When the workgroup holds a whole number of 2x2x2 blocks of cells, it
  // takes such blocks, and the two cells on either side of a face inside a
  // block hand each other their traces of that face through LDS.
  static constexpr bool SUB = CPB % 8 == 0;
  // LDS words per cell: u at the points, its three reference gradients, the
  // three gradient fluxes, the value flux (8 n^3), and five face planes per
  // face of the current direction (P, PN, and P and PN interpolated or
  // differentiated along p1; or the four trace planes handed to the partner)
  static constexpr int CELL = 8 * N3 + 10 * N2;
};

// 3D array [z][y][x] of extent N^3: lane t (0..n^2-1) owns line t along `axis`:
//   out[line][q] (+)= sum_m A'[q][m] in[line][m],  A' = A or A^T (row-major N x N)
template <int N, int AXIS, bool TR, bool ACC, typename T>
__device__ __forceinline__ void sweep3(const T* __restrict__ A, const T* in, T* out, int t) {
  constexpr int N2 = N * N;
  constexpr int st = AXIS == 0 ? 1 : (AXIS == 1 ? N : N2);
  const int a = t % N, b = t / N;
  const int base = AXIS == 0 ? t * N : (AXIS == 1 ? b * N2 + a : t);
  T v[N];
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] = in[base + m * st];
#pragma unroll
  for (int q = 0; q < N; ++q) {
    T s = ACC ? out[base + q * st] : T(0);
#pragma unroll
    for (int m = 0; m < N; ++m) s = fma(TR ? A[m * N + q] : A[q * N + m], v[m], s);
    out[base + q * st] = s;
  }
}

// node index of face-plane entry (p1 along t1, p2 along t2) of the plane at
// coordinate e along direction d
template <int N>
__device__ __forceinline__ int fnode(int d, int e, int p1, int p2) {
  if (d == 0) return (p2 * N + p1) * N + e;
  if (d == 1) return (p2 * N + e) * N + p1;
  return (e * N + p2) * N + p1;
}

template <typename T>
__device__ __forceinline__ int plane_index(const MetricGeom<T>& g, int d, int c0, int c1, int c2) {
  if (d == 0) return c2 * g.ny + c1;
  if (d == 1) return c2 * g.nx + c0;
  return c1 * g.nx + c0;
}

// EPI: dst holds x_{k-1} on entry and receives the Chebyshev step
// x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 D^{-1} (b - H x_k), x_k = src, at the store.
template <int N, typename T, bool EPI>
__global__ void __launch_bounds__(MetShape<N>::THREADS) k_sipg_metric_apply(const T* __restrict__ src,
                                                                             T* __restrict__ dst, const MetricGeom<T> g,
                                                                             double* __restrict__ partials,
                                                                             const int* stop, const ChebEpi<T> epi) {
  if (stop && *stop) return;
  using M = MetShape<N>;
  constexpr int N2 = M::N2, N3 = M::N3;
  constexpr bool SUB = M::SUB;
  __shared__ T s_cells[M::CPB * M::CELL];
  __shared__ double s_red[3 * M::WAVES];
  __shared__ T s_sd[2 * N2];   // S and D: the face-plane steps read a row per lane
  const int tid = threadIdx.x;
  const int lane = tid & 63, w = tid >> 6;
  const int cw = lane / N2;
  const int t = lane - cw * N2;
  const int lc = w * M::CPW + (cw < M::CPW ? cw : 0);   // the cell's slot in the workgroup
  const int nd[3] = {g.nx, g.ny, g.nz};
  int c[3], cell;
  bool act;
  if constexpr (SUB) {
    // workgroup b takes the 2x2x2 blocks b * CPB / 8 ... (x fastest)
    const int bx = (g.nx + 1) >> 1, by = (g.ny + 1) >> 1, bz = (g.nz + 1) >> 1;
    const int blk = blockIdx.x * (M::CPB / 8) + (lc >> 3), j = lc & 7;
    const int sx = blk % bx, sy = (blk / bx) % by, sz = blk / (bx * by);
    c[0] = 2 * sx + (j & 1);
    c[1] = 2 * sy + ((j >> 1) & 1);
    c[2] = 2 * sz + (j >> 2);
    act = cw < M::CPW && sz < bz && c[0] < g.nx && c[1] < g.ny && c[2] < g.nz;
    cell = act ? (c[2] * g.ny + c[1]) * g.nx + c[0] : 0;
  } else {
    cell = blockIdx.x * M::CPB + lc;
    act = cw < M::CPW && cell < g.nx * g.ny * g.nz;
    c[0] = cell % g.nx;
    c[1] = (cell / g.nx) % g.ny;
    c[2] = cell / (g.nx * g.ny);
  }
  T* sA = s_cells + lc * M::CELL;   // u at the Gauss points
  T* sB = sA + N3;           // 3 n^3: reference gradients at the points
  T* sG = sA + 4 * N3;       // 3 n^3: gradient fluxes (nodal u on entry)
  T* sC = sA + 7 * N3;       // value flux
  T* sF = sA + 8 * N3;       // face planes of the current direction, five per face
  const T* S = g.tab + MTab{N}.S();
  const T* D = g.tab + MTab{N}.D();
  for (int i = tid; i < 2 * N2; i += M::THREADS) s_sd[i] = i < N2 ? S[i] : D[i - N2];
  __syncthreads();
  const T* Sl = s_sd;
  const T* Dl = s_sd + N2;
  const T* Dg = g.tab + MTab{N}.Dg();
  const T* g0 = g.tab + MTab{N}.g0();
  const T* g1 = g.tab + MTab{N}.g1();
  const T* E0 = g.tab + MTab{N}.e0();
  const T* E1 = g.tab + MTab{N}.e1();
  double pq = 0.0, sq = 0.0, sp = 0.0;
  const int p1 = t % N, p2 = t / N;
  // ---- every global load of this cell is issued up front, so that their
  // latencies overlap the cell integral (in fp64 the cell and face metric
  // are loaded where they are used: hoisting them too would cost the
  // registers of a second wavefront per SIMD)
  constexpr bool kHoist = sizeof(T) == 4;
  // neighbour face lines: up front unless that alone exhausts the fp64
  // register file (n >= 7), where they are read per face
  constexpr bool kHoistNb = sizeof(T) == 4 || N <= 6;
  T uo[N], cmv[7][N];
  int nbc[6];
  bool ownL[6];
  const T* fmp[6];
  T ftau[6], nbv[6][N], fmv[6][7];
  if (act) {
    const int stride[3] = {1, g.nx, g.nx * g.ny};
    const T* cm = g.cm + static_cast<int64_t>(cell) * 7 * N3;
#pragma unroll
    for (int m = 0; m < N; ++m) uo[m] = src[cell * N3 + t + m * N2];
    if constexpr (kHoist) {
#pragma unroll
      for (int k = 0; k < 7; ++k)
#pragma unroll
        for (int m = 0; m < N; ++m) cmv[k][m] = cm[k * N3 + t + m * N2];
    }
#pragma unroll
    for (int f = 0; f < 6; ++f) {
      const int d = f >> 1, s = f & 1;
      int cn = c[d] + (s ? 1 : -1);
      nbc[f] = -1;
      if (cn < 0 || cn >= nd[d]) {
        if (g.per[d]) cn = cn < 0 ? nd[d] - 1 : 0;
        else cn = -1;
      }
      if (cn >= 0) nbc[f] = cell + (cn - c[d]) * stride[d];
      if (s == 1) {
        fmp[f] = g.fm + (static_cast<int64_t>(cell) * 3 + d) * 7 * N2;
        ftau[f] = g.ftau[cell * 3 + d];
        ownL[f] = true;
      } else if (nbc[f] >= 0) {
        fmp[f] = g.fm + (static_cast<int64_t>(nbc[f]) * 3 + d) * 7 * N2;
        ftau[f] = g.ftau[nbc[f] * 3 + d];
        ownL[f] = false;
      } else {
        const int pi = plane_index(g, d, c[0], c[1], c[2]);
        fmp[f] = g.lm + (static_cast<int64_t>(g.lbase[d]) + pi) * 7 * N2;
        ftau[f] = g.ltau[g.lbase[d] + pi];
        ownL[f] = true;
      }
      if constexpr (kHoist) {
#pragma unroll
        for (int k = 0; k < 7; ++k) fmv[f][k] = gld(fmp[f] + k * N2 + t);
      }
      // neighbour face lines (not across the face shared with the block
      // partner: those traces come through LDS)
      const bool partner = SUB && (c[d] ^ 1) < nd[d] && s == 1 - (c[d] & 1);
      if (kHoistNb && nbc[f] >= 0 && !partner) {
        const T* un = src + static_cast<int64_t>(nbc[f]) * N3;
#pragma unroll
        for (int m = 0; m < N; ++m) nbv[f][m] = un[fnode<N>(d, m, p1, p2)];
      } else {
#pragma unroll
        for (int m = 0; m < N; ++m) nbv[f][m] = T(0);
      }
    }
    // ---- values and reference gradients at the Gauss points
#pragma unroll
    for (int m = 0; m < N; ++m) sG[t + m * N2] = uo[m];
    wave_sync();
    sweep3<N, 0, false, false>(S, sG, sC, t);
    wave_sync();
    sweep3<N, 1, false, false>(S, sC, sG + N3, t);
    wave_sync();
    sweep3<N, 2, false, false>(S, sG + N3, sA, t);   // sA = u at the points
    wave_sync();
    sweep3<N, 0, false, false>(Dg, sA, sB, t);
    sweep3<N, 1, false, false>(Dg, sA, sB + N3, t);
    sweep3<N, 2, false, false>(Dg, sA, sB + 2 * N3, t);
    wave_sync();
    // ---- cell integrand: nu (w detJ J^-1 J^-T) grad u and mu w detJ u at every point
    if constexpr (!kHoist) {
#pragma unroll
      for (int k = 0; k < 7; ++k)
#pragma unroll
        for (int m = 0; m < N; ++m) cmv[k][m] = cm[k * N3 + t + m * N2];
    }
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const int q = t + m * N2;
      const T gx = sB[q], gy = sB[N3 + q], gz = sB[2 * N3 + q];
      sG[q] = g.nu * (cmv[0][m] * gx + cmv[1][m] * gy + cmv[2][m] * gz);
      sG[N3 + q] = g.nu * (cmv[1][m] * gx + cmv[3][m] * gy + cmv[4][m] * gz);
      sG[2 * N3 + q] = g.nu * (cmv[2][m] * gx + cmv[4][m] * gy + cmv[5][m] * gz);
      sC[q] = g.mu * cmv[6][m] * sA[q];
    }
    wave_sync();
  }
  // ---- faces.  Lane t is face point (p1, p2).  Own traces are the values
  // of the Gauss-point data extrapolated along the normal line (exact: every
  // field is a polynomial of degree < n along it); the face terms go back
  // through the transpose of that extrapolation into the point fluxes, so
  // the transposed cell sweeps below lift them.  The two faces of a direction
  // share the normal lines: both own traces come from one pass over the line
  // and both face terms go back in one read-modify-write of it.  A
  // neighbour's traces (value, d/dt1, d/dt2, d/dn at the face point) are
  // the own traces of the partner cell across a face inside a 2x2x2 block;
  // otherwise they come from the neighbour's nodal face plane P and its
  // normal-derivative plane PN, interpolated (S) or differentiated (D) along
  // p1, then along p2, each lane forming its own point of every plane.  The
  // workgroup barriers of the block exchange are reached by every thread.
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    T uf[2] = {T(0), T(0)}, gf[2][3] = {{T(0), T(0), T(0)}, {T(0), T(0), T(0)}};
    if (act) {
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const int q = fnode<N>(d, m, p1, p2);
        const T a = sA[q], b0 = sB[q], b1 = sB[N3 + q], b2 = sB[2 * N3 + q];
        uf[0] = fma(E0[m], a, uf[0]);
        uf[1] = fma(E1[m], a, uf[1]);
        gf[0][0] = fma(E0[m], b0, gf[0][0]);
        gf[1][0] = fma(E1[m], b0, gf[1][0]);
        gf[0][1] = fma(E0[m], b1, gf[0][1]);
        gf[1][1] = fma(E1[m], b1, gf[1][1]);
        gf[0][2] = fma(E0[m], b2, gf[0][2]);
        gf[1][2] = fma(E1[m], b2, gf[1][2]);
      }
    }
    // the face shared with the block partner (-1: none)
    int fx = -1;
    if constexpr (SUB) {
      if (act && (c[d] ^ 1) < nd[d]) fx = 1 - (c[d] & 1);
    }
    T nbt[2][4];
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int k = 0; k < 4; ++k) nbt[s][k] = T(0);
    if (act) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * d + s;
        T* F = sF + 5 * s * N2;
        if (s == fx) {
          F[t] = uf[s];
          F[N2 + t] = gf[s][0];
          F[2 * N2 + t] = gf[s][1];
          F[3 * N2 + t] = gf[s][2];
        } else if (nbc[f] >= 0) {
          if constexpr (!kHoistNb) {
            const T* un = src + static_cast<int64_t>(nbc[f]) * N3;
#pragma unroll
            for (int m = 0; m < N; ++m) nbv[f][m] = un[fnode<N>(d, m, p1, p2)];
          }
          const T* gn = s ? g0 : g1;      // normal derivative row at the neighbour's face
          T dnn = T(0);
#pragma unroll
          for (int m = 0; m < N; ++m) dnn = fma(gn[m], nbv[f][m], dnn);
          F[t] = nbv[f][s ? 0 : N - 1];
          F[N2 + t] = dnn;
        }
      }
    }
    // (the partner is in this wavefront when 2^d < cells per wavefront)
    if (SUB && (1 << d) >= M::CPW) __syncthreads();
    else wave_sync();
    if (act) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        T* F = sF + 5 * s * N2;
        if (s == fx) {
          const T* X = s_cells + (lc ^ (1 << d)) * M::CELL + 8 * N3 + 5 * (1 - s) * N2;
          const T gx[3] = {X[N2 + t], X[2 * N2 + t], X[3 * N2 + t]};
          nbt[s][0] = X[t];
          nbt[s][1] = gx[t1];
          nbt[s][2] = gx[t2];
          nbt[s][3] = gx[d];
        } else if (nbc[2 * d + s] >= 0) {
          const T* P = F + p2 * N;
          const T* PN = F + N2 + p2 * N;
          T sp = T(0), dp = T(0), spn = T(0);
#pragma unroll
          for (int m = 0; m < N; ++m) {
            const T a = P[m], b = PN[m];
            sp = fma(Sl[p1 * N + m], a, sp);
            dp = fma(Dl[p1 * N + m], a, dp);
            spn = fma(Sl[p1 * N + m], b, spn);
          }
          F[2 * N2 + t] = sp;
          F[3 * N2 + t] = dp;
          F[4 * N2 + t] = spn;
        }
      }
    }
    wave_sync();
    if (act) {
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        if (s != fx && nbc[2 * d + s] >= 0) {
          const T* F = sF + 5 * s * N2;
          const T* SP = F + 2 * N2 + p1;
          const T* DP = F + 3 * N2 + p1;
          const T* SPN = F + 4 * N2 + p1;
#pragma unroll
          for (int m = 0; m < N; ++m) {
            const T a = SP[m * N], b = DP[m * N], c2 = SPN[m * N];
            const T sm = Sl[p2 * N + m];
            nbt[s][0] = fma(sm, a, nbt[s][0]);
            nbt[s][1] = fma(sm, b, nbt[s][1]);
            nbt[s][2] = fma(Dl[p2 * N + m], a, nbt[s][2]);
            nbt[s][3] = fma(sm, c2, nbt[s][3]);
          }
        }
      }
      T fvs[2], fgs[2][3];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * d + s;
        const int nb = nbc[f];
        if constexpr (!kHoist) {
#pragma unroll
          for (int k = 0; k < 7; ++k) fmv[f][k] = gld(fmp[f] + k * N2 + t);
        }
        const bool own_is_L = ownL[f];
        const T tau = ftau[f] * g.pen;
        const T wdA = fmv[f][0];
        T vo[3], vn[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          vo[k] = own_is_L ? fmv[f][1 + k] : fmv[f][4 + k];
          vn[k] = own_is_L ? fmv[f][4 + k] : fmv[f][1 + k];
        }
        const T uo_f = uf[s];
        const T ano = gf[s][0] * vo[0] + gf[s][1] * vo[1] + gf[s][2] * vo[2];
        T fv, fgc;
        if (nb >= 0) {
          T gnb[3];
          gnb[d] = nbt[s][3];
          gnb[t1] = nbt[s][1];
          gnb[t2] = nbt[s][2];
          const T un = nbt[s][0];
          const T ann = gnb[0] * vn[0] + gnb[1] * vn[1] + gnb[2] * vn[2];
          const T jump = own_is_L ? uo_f - un : un - uo_f;
          const T avg = T(0.5) * (ano + ann);
          fv = own_is_L ? (-avg + tau * jump * wdA) : (avg - tau * jump * wdA);
          fgc = T(-0.5) * jump;
        } else {
          // Dirichlet face; a homogeneous Neumann face adds nothing
          const T bw = ((g.neu >> f) & 1) ? T(0) : T(1);
          fv = bw * (-ano + T(2) * tau * uo_f * wdA);
          fgc = -bw * uo_f;
        }
        fvs[s] = fv * g.nu;
        fgc *= g.nu;
#pragma unroll
        for (int k = 0; k < 3; ++k) fgs[s][k] = fgc * vo[k];
      }
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const int q = fnode<N>(d, m, p1, p2);
        sC[q] = fma(E1[m], fvs[1], fma(E0[m], fvs[0], sC[q]));
        sG[q] = fma(E1[m], fgs[1][0], fma(E0[m], fgs[0][0], sG[q]));
        sG[N3 + q] = fma(E1[m], fgs[1][1], fma(E0[m], fgs[0][1], sG[N3 + q]));
        sG[2 * N3 + q] = fma(E1[m], fgs[1][2], fma(E0[m], fgs[0][2], sG[2 * N3 + q]));
      }
    }
    // the partner's reads of this cell's planes end before the next direction writes them
    if (SUB && (1 << d) >= M::CPW) __syncthreads();
    else wave_sync();
  }
  if (act) {
    // ---- transposed sweeps: sC += sum_d Dg_d^T sG_d, then S^T in every direction
    T eb[N], ed[N], ep[N];
    if constexpr (EPI) {   // issued before the sweeps so that their latency overlaps them
#pragma unroll
      for (int m = 0; m < N; ++m) {
        const int64_t at = static_cast<int64_t>(cell) * N3 + t + m * N2;
        eb[m] = epi.b[at];
        ed[m] = epi.dinv[at];
        ep[m] = epi.prev_zero ? T(0) : dst[at];
      }
    }
    sweep3<N, 0, true, true>(Dg, sG, sC, t);
    wave_sync();
    sweep3<N, 1, true, true>(Dg, sG + N3, sC, t);
    wave_sync();
    sweep3<N, 2, true, true>(Dg, sG + 2 * N3, sC, t);
    wave_sync();
    sweep3<N, 2, true, false>(S, sC, sA, t);
    wave_sync();
    sweep3<N, 1, true, false>(S, sA, sB, t);
    wave_sync();
    sweep3<N, 0, true, false>(S, sB, sC, t);
    wave_sync();
#pragma unroll
    for (int m = 0; m < N; ++m) {
      const int e = t + m * N2;
      T v = sC[e];
      if constexpr (EPI) v = fma(epi.c2 * ed[m], eb[m] - v, fma(epi.c1, uo[m] - ep[m], uo[m]));
      dst[cell * N3 + e] = v;
      if (partials) {
        pq += static_cast<double>(uo[m]) * v;
        sq += v;
        sp += uo[m];
      }
    }
  }
  if (partials) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      pq += __shfl_down(pq, o, 64);
      sq += __shfl_down(sq, o, 64);
      sp += __shfl_down(sp, o, 64);
    }
    if (lane == 0) {
      s_red[3 * w] = pq;
      s_red[3 * w + 1] = sq;
      s_red[3 * w + 2] = sp;
    }
    __syncthreads();
    if (tid == 0) {
      double x = 0, y = 0, z = 0;
      for (int k = 0; k < M::WAVES; ++k) {
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

// Diagonal of the operator: one thread per DoF, direct quadrature of the
// cell term and of the own-side face terms of the faces the node lies on.
template <int N, typename TO>
__global__ void __launch_bounds__(256) k_sipg_metric_diag(TO* __restrict__ diag, const MetricGeom<double> g) {
  constexpr int N2 = N * N, N3 = N2 * N;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t ncells = static_cast<int64_t>(g.nx) * g.ny * g.nz;
  if (gid >= ncells * N3) return;
  const int cell = static_cast<int>(gid / N3);
  const int loc = static_cast<int>(gid - static_cast<int64_t>(cell) * N3);
  const int idx[3] = {loc % N, (loc / N) % N, loc / N2};
  const int c[3] = {cell % g.nx, (cell / g.nx) % g.ny, cell / (g.nx * g.ny)};
  const int nd[3] = {g.nx, g.ny, g.nz};
  const double* S = g.tab + MTab{N}.S();
  const double* D = g.tab + MTab{N}.D();
  const double* g0 = g.tab + MTab{N}.g0();
  const double* g1 = g.tab + MTab{N}.g1();
  const double* cm = g.cm + static_cast<int64_t>(cell) * 7 * N3;
  double acc = 0.0;
  for (int qz = 0; qz < N; ++qz)
    for (int qy = 0; qy < N; ++qy)
      for (int qx = 0; qx < N; ++qx) {
        const int q = (qz * N + qy) * N + qx;
        const double sx = S[qx * N + idx[0]], sy = S[qy * N + idx[1]], sz = S[qz * N + idx[2]];
        const double gx = D[qx * N + idx[0]] * sy * sz, gy = sx * D[qy * N + idx[1]] * sz,
                     gz = sx * sy * D[qz * N + idx[2]];
        const double G00 = cm[q], G01 = cm[N3 + q], G02 = cm[2 * N3 + q];
        const double G11 = cm[3 * N3 + q], G12 = cm[4 * N3 + q], G22 = cm[5 * N3 + q], m = cm[6 * N3 + q];
        const double phi = sx * sy * sz;
        acc += g.nu * (gx * (G00 * gx + G01 * gy + G02 * gz) + gy * (G01 * gx + G11 * gy + G12 * gz) +
                       gz * (G02 * gx + G12 * gy + G22 * gz)) +
               g.mu * m * phi * phi;
      }
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    for (int s = 0; s < 2; ++s) {
      if (idx[d] != (s ? N - 1 : 0)) continue;          // the node is not on this face
      int cn = c[d] + (s ? 1 : -1);
      bool dir = false;
      if (cn < 0 || cn >= nd[d]) {
        if (g.per[d]) cn = cn < 0 ? nd[d] - 1 : 0;
        else dir = true;
      }
      if (dir && ((g.neu >> (2 * d + s)) & 1)) continue;   // homogeneous Neumann face: no term
      const double* fm;
      double tau;
      bool own_is_L;
      if (s == 1) {
        fm = g.fm + (static_cast<int64_t>(cell) * 3 + d) * 7 * N2;
        tau = g.ftau[cell * 3 + d];
        own_is_L = true;
      } else if (!dir) {
        const int nb = cell + (cn - c[d]) * (d == 0 ? 1 : (d == 1 ? g.nx : g.nx * g.ny));
        fm = g.fm + (static_cast<int64_t>(nb) * 3 + d) * 7 * N2;
        tau = g.ftau[nb * 3 + d];
        own_is_L = false;
      } else {
        const int pi = plane_index(g, d, c[0], c[1], c[2]);
        fm = g.lm + (static_cast<int64_t>(g.lbase[d]) + pi) * 7 * N2;
        tau = g.ltau[g.lbase[d] + pi];
        own_is_L = true;
      }
      tau *= g.pen;
      const double gsd = (s ? g1 : g0)[idx[d]];
      const double fac = dir ? 2.0 : 1.0;
      const double sgn = own_is_L ? -1.0 : 1.0;    // -(grad phi.n_out, phi): n_out = n for L, -n for R
      for (int q2 = 0; q2 < N; ++q2)
        for (int q1 = 0; q1 < N; ++q1) {
          const int p = q2 * N + q1;
          const double a1 = S[q1 * N + idx[t1]], a2 = S[q2 * N + idx[t2]];
          const double phi = a1 * a2;
          double gh[3];
          gh[d] = gsd * phi;
          gh[t1] = D[q1 * N + idx[t1]] * a2;
          gh[t2] = a1 * D[q2 * N + idx[t2]];
          const double* v = fm + (own_is_L ? 1 : 4) * N2;
          const double gv = gh[0] * v[p] + gh[1] * v[N2 + p] + gh[2] * v[2 * N2 + p];
          acc += g.nu * fac * (sgn * gv * phi + tau * fm[p] * phi * phi);
        }
    }
  }
  diag[gid] = static_cast<TO>(acc);
}

// Geometry fill: one thread per (cell, entry).  J = Sh diag(h) on every cell,
// Sh the constant lattice matrix (identity for plain boxes).
struct FillArgs {
  MetricGeom<double> g;
  const double* x0[3];
  const double* h[3];
  double shinv[9];   // Sh^{-1}, row-major
  double shdet;      // det Sh
  double k1sq;       // (k+1)^2
  const double* wq;  // Gauss weights (N)
};

__device__ __forceinline__ void cell_jinv(const FillArgs& a, const int c[3], double Jinv[9], double& detJ) {
  double hv[3];
  for (int d = 0; d < 3; ++d) hv[d] = a.h[d][c[d]];
  // J^{-1} = diag(1/h) Sh^{-1}
  for (int r = 0; r < 3; ++r)
    for (int col = 0; col < 3; ++col) Jinv[r * 3 + col] = a.shinv[r * 3 + col] / hv[r];
  detJ = fabs(a.shdet) * hv[0] * hv[1] * hv[2];
}

__device__ __forceinline__ double cell_tau(const FillArgs& a, const int c[3]) {
  double Jinv[9], detJ;
  cell_jinv(a, c, Jinv, detJ);
  const int nd[3] = {a.g.nx, a.g.ny, a.g.nz};
  double t = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double rn = sqrt(Jinv[d * 3] * Jinv[d * 3] + Jinv[d * 3 + 1] * Jinv[d * 3 + 1] + Jinv[d * 3 + 2] * Jinv[d * 3 + 2]);
    double wsum = 1.0;   // two interior faces, half each
    if (!a.g.per[d]) {
      if (nd[d] == 1) wsum = 2.0;
      else if (c[d] == 0 || c[d] == nd[d] - 1) wsum = 1.5;
    }
    t += wsum * rn;      // A_f / V = |J^{-T} e_d|
  }
  return a.k1sq * t;
}

template <int N>
__global__ void __launch_bounds__(256) k_metric_fill_cells(FillArgs a, double* cm) {
  constexpr int N3 = N * N * N;
  const int64_t ncells = static_cast<int64_t>(a.g.nx) * a.g.ny * a.g.nz;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= ncells * N3) return;
  const int cell = static_cast<int>(gid / N3);
  const int q = static_cast<int>(gid - static_cast<int64_t>(cell) * N3);
  const int c[3] = {cell % a.g.nx, (cell / a.g.nx) % a.g.ny, cell / (a.g.nx * a.g.ny)};
  double Jinv[9], detJ;
  cell_jinv(a, c, Jinv, detJ);
  const double w = a.wq[q % N] * a.wq[(q / N) % N] * a.wq[q / (N * N)] * detJ;
  double G[6];
  int k = 0;
  for (int r = 0; r < 3; ++r)
    for (int col = r; col < 3; ++col) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += Jinv[r * 3 + m] * Jinv[col * 3 + m];
      G[k++] = w * s;
    }
  double* out = cm + static_cast<int64_t>(cell) * 7 * N3;
  for (int e = 0; e < 6; ++e) out[e * N3 + q] = G[e];
  out[6 * N3 + q] = w;
}

// high faces (cell, d): entries 7 x N2; low boundary faces in non-periodic directions
template <int N>
__global__ void __launch_bounds__(256) k_metric_fill_faces(FillArgs a, double* fm, double* ftau, double* lm,
                                                           double* ltau) {
  constexpr int N2 = N * N;
  const int64_t ncells = static_cast<int64_t>(a.g.nx) * a.g.ny * a.g.nz;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= ncells * 6 * N2) return;
  const int p = static_cast<int>(gid % N2);
  const int64_t fc = gid / N2;
  const int f = static_cast<int>(fc % 6);
  const int cell = static_cast<int>(fc / 6);
  const int d = f >> 1, s = f & 1;
  const int c[3] = {cell % a.g.nx, (cell / a.g.nx) % a.g.ny, cell / (a.g.nx * a.g.ny)};
  const int nd[3] = {a.g.nx, a.g.ny, a.g.nz};
  int cn = c[d] + (s ? 1 : -1);
  bool dir = false;
  if (cn < 0 || cn >= nd[d]) {
    if (a.g.per[d]) cn = cn < 0 ? nd[d] - 1 : 0;
    else dir = true;
  }
  if (s == 0 && !dir) return;            // an interior low face is stored as the neighbour's high face
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  (void)t1;
  (void)t2;
  double Jl[9], detl;
  cell_jinv(a, c, Jl, detl);
  double rn = 0.0;
  for (int m = 0; m < 3; ++m) rn += Jl[d * 3 + m] * Jl[d * 3 + m];
  rn = sqrt(rn);
  double n[3];
  for (int m = 0; m < 3; ++m) n[m] = (s ? 1.0 : -1.0) * Jl[d * 3 + m] / rn;   // outward from this cell
  const double wdA = a.wq[p % N] * a.wq[p / N] * detl * rn;
  double vL[3], vR[3] = {0.0, 0.0, 0.0};
  for (int r = 0; r < 3; ++r) vL[r] = wdA * (Jl[r * 3] * n[0] + Jl[r * 3 + 1] * n[1] + Jl[r * 3 + 2] * n[2]);
  double tau = cell_tau(a, c);
  if (!dir) {
    int cr[3] = {c[0], c[1], c[2]};
    cr[d] = cn;
    double Jr[9], detr;
    cell_jinv(a, cr, Jr, detr);
    for (int r = 0; r < 3; ++r) vR[r] = wdA * (Jr[r * 3] * n[0] + Jr[r * 3 + 1] * n[1] + Jr[r * 3 + 2] * n[2]);
    const double tr = cell_tau(a, cr);
    tau = tau > tr ? tau : tr;
  }
  double* out;
  if (s == 1) {
    out = fm + (static_cast<int64_t>(cell) * 3 + d) * 7 * N2;
    if (p == 0) ftau[cell * 3 + d] = tau;
  } else {
    const int pi = plane_index(a.g, d, c[0], c[1], c[2]);
    out = lm + (static_cast<int64_t>(a.g.lbase[d]) + pi) * 7 * N2;
    if (p == 0) ltau[a.g.lbase[d] + pi] = tau;
  }
  out[p] = wdA;
  for (int r = 0; r < 3; ++r) {
    out[(1 + r) * N2 + p] = vL[r];
    out[(4 + r) * N2 + p] = vR[r];
  }
}

// Curved (iso-parametric) geometry fill, with the closed-form Jacobian of
// curv_map.h.  ctab: GLL nodes, S and D rows at the Gauss points, l(0), l(1),
// l'(0), l'(1), Gauss weights (n each / n x n).
struct CurvArgs {
  MetricGeom<double> g;
  CurvMap map;
  double k1sq;
  const double* ctab;
  const double* taue;   // per-cell (k+1)^2 (A_int/2 + A_bnd) / V (faces kernel)
};

struct CurvTabs {
  int n;
  __device__ const double* nodes(const double* t) const { return t; }
  __device__ const double* S(const double* t) const { return t + n; }
  __device__ const double* D(const double* t) const { return t + n + n * n; }
  __device__ const double* E(const double* t, int s) const { return t + n + 2 * n * n + s * n; }
  __device__ const double* G(const double* t, int s) const { return t + 3 * n + 2 * n * n + s * n; }
  __device__ const double* W(const double* t) const { return t + 5 * n + 2 * n * n; }
};

// J (row-major J[r*3+d]) of cell c at the reference point whose per-direction rows are (val[e], der[e])
template <int N>
__device__ __forceinline__ void curv_jac(const CurvArgs& a, const int c[3], const double* const val[3],
                                         const double* const der[3], double J[9]) {
  curv_jac_at<N>(a.map, c, val, der, J);
}

__device__ __forceinline__ double inv3(const double J[9], double Ji[9]) {
  const double c00 = J[4] * J[8] - J[5] * J[7], c01 = J[5] * J[6] - J[3] * J[8], c02 = J[3] * J[7] - J[4] * J[6];
  const double det = J[0] * c00 + J[1] * c01 + J[2] * c02;
  const double r = 1.0 / det;
  Ji[0] = c00 * r;
  Ji[1] = (J[2] * J[7] - J[1] * J[8]) * r;
  Ji[2] = (J[1] * J[5] - J[2] * J[4]) * r;
  Ji[3] = c01 * r;
  Ji[4] = (J[0] * J[8] - J[2] * J[6]) * r;
  Ji[5] = (J[2] * J[3] - J[0] * J[5]) * r;
  Ji[6] = c02 * r;
  Ji[7] = (J[1] * J[6] - J[0] * J[7]) * r;
  Ji[8] = (J[0] * J[4] - J[1] * J[3]) * r;
  return det;
}

// rows of point index qe (0..N-1: Gauss point) or end point s (N + s) along one direction
template <int N>
__device__ __forceinline__ void curv_rows(const CurvArgs& a, int qe, const double*& val, const double*& der) {
  const CurvTabs T{N};
  if (qe < N) {
    val = T.S(a.ctab) + qe * N;
    der = T.D(a.ctab) + qe * N;
  } else {
    val = T.E(a.ctab, qe - N);
    der = T.G(a.ctab, qe - N);
  }
}

// face f = 2d+s of cell c at tangential Gauss indices (p1, p2): J^{-1}, det, the row d of J^{-1}
template <int N>
__device__ __forceinline__ double curv_face_jinv(const CurvArgs& a, const int c[3], int d, int s, int p1, int p2,
                                                 double Ji[9]) {
  const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
  int qi[3];
  qi[d] = N + s;
  qi[t1] = p1;
  qi[t2] = p2;
  const double* val[3];
  const double* der[3];
#pragma unroll
  for (int e = 0; e < 3; ++e) curv_rows<N>(a, qi[e], val[e], der[e]);
  double J[9];
  curv_jac<N>(a, c, val, der, J);
  return fabs(inv3(J, Ji));
}

// tau_e / s of every cell: (k+1)^2 (sum over faces of w_f A_f) / V, w_f = 1/2 inside, 1 on the boundary
template <int N>
__global__ void __launch_bounds__(256) k_curved_tau(CurvArgs a, double* taue) {
  const int64_t ncells = static_cast<int64_t>(a.g.nx) * a.g.ny * a.g.nz;
  const int64_t cell = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (cell >= ncells) return;
  const int c[3] = {static_cast<int>(cell % a.g.nx), static_cast<int>((cell / a.g.nx) % a.g.ny),
                    static_cast<int>(cell / (static_cast<int64_t>(a.g.nx) * a.g.ny))};
  const int nd[3] = {a.g.nx, a.g.ny, a.g.nz};
  const double* w = CurvTabs{N}.W(a.ctab);
  double vol = 0.0;
  for (int q = 0; q < N * N * N; ++q) {
    const int qi[3] = {q % N, (q / N) % N, q / (N * N)};
    const double* val[3];
    const double* der[3];
    for (int e = 0; e < 3; ++e) curv_rows<N>(a, qi[e], val[e], der[e]);
    double J[9], Ji[9];
    curv_jac<N>(a, c, val, der, J);
    vol += w[qi[0]] * w[qi[1]] * w[qi[2]] * fabs(inv3(J, Ji));
  }
  double area = 0.0;
  for (int f = 0; f < 6; ++f) {
    const int d = f >> 1, s = f & 1;
    const bool bnd = !a.g.per[d] && (s ? c[d] == nd[d] - 1 : c[d] == 0);
    double A = 0.0;
    for (int p = 0; p < N * N; ++p) {
      double Ji[9];
      const double det = curv_face_jinv<N>(a, c, d, s, p % N, p / N, Ji);
      const double rn = sqrt(Ji[d * 3] * Ji[d * 3] + Ji[d * 3 + 1] * Ji[d * 3 + 1] + Ji[d * 3 + 2] * Ji[d * 3 + 2]);
      A += w[p % N] * w[p / N] * det * rn;
    }
    area += (bnd ? 1.0 : 0.5) * A;
  }
  taue[cell] = a.k1sq * area / vol;
}

template <int N>
__global__ void __launch_bounds__(256) k_curved_fill_cells(CurvArgs a, double* cm) {
  constexpr int N3 = N * N * N;
  const int64_t ncells = static_cast<int64_t>(a.g.nx) * a.g.ny * a.g.nz;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= ncells * N3) return;
  const int64_t cell = gid / N3;
  const int q = static_cast<int>(gid - cell * N3);
  const int c[3] = {static_cast<int>(cell % a.g.nx), static_cast<int>((cell / a.g.nx) % a.g.ny),
                    static_cast<int>(cell / (static_cast<int64_t>(a.g.nx) * a.g.ny))};
  const int qi[3] = {q % N, (q / N) % N, q / (N * N)};
  const double* val[3];
  const double* der[3];
  for (int e = 0; e < 3; ++e) curv_rows<N>(a, qi[e], val[e], der[e]);
  double J[9], Ji[9];
  curv_jac<N>(a, c, val, der, J);
  const double* wq = CurvTabs{N}.W(a.ctab);
  const double w = wq[qi[0]] * wq[qi[1]] * wq[qi[2]] * fabs(inv3(J, Ji));
  double G[6];
  int k = 0;
  for (int r = 0; r < 3; ++r)
    for (int col = r; col < 3; ++col) {
      double s = 0.0;
      for (int m = 0; m < 3; ++m) s += Ji[r * 3 + m] * Ji[col * 3 + m];
      G[k++] = w * s;
    }
  double* out = cm + cell * 7 * N3;
  for (int e = 0; e < 6; ++e) out[e * N3 + q] = G[e];
  out[6 * N3 + q] = w;
}

// high faces (cell, d) and low boundary faces, as k_metric_fill_faces, with the
// Jacobians of both cells at the face point
template <int N>
__global__ void __launch_bounds__(256) k_curved_fill_faces(CurvArgs a, double* fm, double* ftau, double* lm,
                                                           double* ltau) {
  constexpr int N2 = N * N;
  const int64_t ncells = static_cast<int64_t>(a.g.nx) * a.g.ny * a.g.nz;
  const int64_t gid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (gid >= ncells * 6 * N2) return;
  const int p = static_cast<int>(gid % N2);
  const int64_t fc = gid / N2;
  const int f = static_cast<int>(fc % 6);
  const int64_t cell = fc / 6;
  const int d = f >> 1, s = f & 1;
  const int c[3] = {static_cast<int>(cell % a.g.nx), static_cast<int>((cell / a.g.nx) % a.g.ny),
                    static_cast<int>(cell / (static_cast<int64_t>(a.g.nx) * a.g.ny))};
  const int nd[3] = {a.g.nx, a.g.ny, a.g.nz};
  int cn = c[d] + (s ? 1 : -1);
  bool dir = false;
  if (cn < 0 || cn >= nd[d]) {
    if (a.g.per[d]) cn = cn < 0 ? nd[d] - 1 : 0;
    else dir = true;
  }
  if (s == 0 && !dir) return;            // an interior low face is stored as the neighbour's high face
  const int p1 = p % N, p2 = p / N;
  double Jl[9];
  const double detl = curv_face_jinv<N>(a, c, d, s, p1, p2, Jl);
  double rn = 0.0;
  for (int m = 0; m < 3; ++m) rn += Jl[d * 3 + m] * Jl[d * 3 + m];
  rn = sqrt(rn);
  double n[3];
  for (int m = 0; m < 3; ++m) n[m] = (s ? 1.0 : -1.0) * Jl[d * 3 + m] / rn;   // outward from this cell
  const double* wq = CurvTabs{N}.W(a.ctab);
  const double wdA = wq[p1] * wq[p2] * detl * rn;
  double vL[3], vR[3] = {0.0, 0.0, 0.0};
  for (int r = 0; r < 3; ++r) vL[r] = wdA * (Jl[r * 3] * n[0] + Jl[r * 3 + 1] * n[1] + Jl[r * 3 + 2] * n[2]);
  double tau = a.taue[cell];
  if (!dir) {
    int cr[3] = {c[0], c[1], c[2]};
    cr[d] = cn;
    double Jr[9];
    curv_face_jinv<N>(a, cr, d, 1 - s, p1, p2, Jr);
    for (int r = 0; r < 3; ++r) vR[r] = wdA * (Jr[r * 3] * n[0] + Jr[r * 3 + 1] * n[1] + Jr[r * 3 + 2] * n[2]);
    const int64_t ncell = cell + static_cast<int64_t>(cn - c[d]) *
                                     (d == 0 ? 1 : (d == 1 ? a.g.nx : static_cast<int64_t>(a.g.nx) * a.g.ny));
    const double tr = a.taue[ncell];
    tau = tau > tr ? tau : tr;
  }
  double* out;
  if (s == 1) {
    out = fm + (cell * 3 + d) * 7 * N2;
    if (p == 0) ftau[cell * 3 + d] = tau;
  } else {
    const int pi = plane_index(a.g, d, c[0], c[1], c[2]);
    out = lm + (static_cast<int64_t>(a.g.lbase[d]) + pi) * 7 * N2;
    if (p == 0) ltau[a.g.lbase[d] + pi] = tau;
  }
  out[p] = wdA;
  for (int r = 0; r < 3; ++r) {
    out[(1 + r) * N2 + p] = vL[r];
    out[(4 + r) * N2 + p] = vR[r];
  }
}

__global__ void __launch_bounds__(256) k_to_f32(const double* __restrict__ a, float* __restrict__ b, int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x)
    b[i] = static_cast<float>(a[i]);
}

}  // namespace

#define DGMF_MET_CASES(X) X(2) X(3) X(4) X(5) X(6) X(7) X(8)

int metric_apply_blocks(int n, int nx, int ny, int nz) {
  const int cpb = 4 * (64 / (n * n));
  if (cpb % 8 == 0) {   // cpb / 8 blocks of 2x2x2 cells per workgroup
    const int64_t blocks = static_cast<int64_t>((nx + 1) / 2) * ((ny + 1) / 2) * ((nz + 1) / 2);
    return static_cast<int>((blocks + cpb / 8 - 1) / (cpb / 8));
  }
  return static_cast<int>((static_cast<int64_t>(nx) * ny * nz + cpb - 1) / cpb);
}

template <typename T, bool EPI>
dgmf_status launch_metric(int n, const MetricGeom<T>& g, const T* src, T* dst, double* partials, const int* stop,
                          const ChebEpi<T>& epi, hipStream_t s) {
  const unsigned blocks = static_cast<unsigned>(metric_apply_blocks(n, g.nx, g.ny, g.nz));
#define X(a)                                                                                                 \
  if (n == a) {                                                                                              \
    hipLaunchKernelGGL((k_sipg_metric_apply<a, T, EPI>), dim3(blocks), dim3(MetShape<a>::THREADS), 0, s, src, \
                       dst, g, partials, stop, epi);                                                         \
    DGMF_LAUNCH_CHECK("k_sipg_metric_apply");                                                                \
    return DGMF_OK;                                                                                          \
  }
  DGMF_MET_CASES(X)
#undef X
  return fail(DGMF_UNSUPPORTED, "metric apply: degree %d not built", n - 1);
}

template <typename T>
dgmf_status launch_sipg_metric_apply(int n, const MetricGeom<T>& g, const T* src, T* dst, double* partials,
                                     const int* stop, hipStream_t s) {
  const ChebEpi<T> none{nullptr, nullptr, T(0), T(0), 1};
  return launch_metric<T, false>(n, g, src, dst, partials, stop, none, s);
}

template <typename T>
dgmf_status launch_sipg_metric_cheb(int n, const MetricGeom<T>& g, const T* xk, T* dst, const ChebEpi<T>& epi,
                                    const int* stop, hipStream_t s) {
  return launch_metric<T, true>(n, g, xk, dst, nullptr, stop, epi, s);
}

template dgmf_status launch_sipg_metric_apply<double>(int, const MetricGeom<double>&, const double*, double*,
                                                      double*, const int*, hipStream_t);
template dgmf_status launch_sipg_metric_apply<float>(int, const MetricGeom<float>&, const float*, float*, double*,
                                                     const int*, hipStream_t);
template dgmf_status launch_sipg_metric_cheb<double>(int, const MetricGeom<double>&, const double*, double*,
                                                     const ChebEpi<double>&, const int*, hipStream_t);
template dgmf_status launch_sipg_metric_cheb<float>(int, const MetricGeom<float>&, const float*, float*,
                                                    const ChebEpi<float>&, const int*, hipStream_t);

dgmf_status launch_to_f32(const double* a, float* b, int64_t n, hipStream_t s) {
  if (n <= 0) return DGMF_OK;
  const int64_t want = (n + 255) / 256;
  const unsigned blocks = static_cast<unsigned>(want < 8192 ? want : 8192);
  hipLaunchKernelGGL(k_to_f32, dim3(blocks), dim3(256), 0, s, a, b, n);
  DGMF_LAUNCH_CHECK("k_to_f32");
  return DGMF_OK;
}

template <typename TO>
dgmf_status launch_sipg_metric_diag(int n, const MetricGeom<double>& g, TO* diag, hipStream_t s) {
  const int64_t total = static_cast<int64_t>(g.nx) * g.ny * g.nz * n * n * n;
  const unsigned blocks = static_cast<unsigned>((total + 255) / 256);
#define X(a)                                                                                   \
  if (n == a) {                                                                                \
    hipLaunchKernelGGL((k_sipg_metric_diag<a, TO>), dim3(blocks), dim3(256), 0, s, diag, g);  \
    DGMF_LAUNCH_CHECK("k_sipg_metric_diag");                                                   \
    return DGMF_OK;                                                                            \
  }
  DGMF_MET_CASES(X)
#undef X
  return fail(DGMF_UNSUPPORTED, "metric diagonal: degree %d not built", n - 1);
}

template dgmf_status launch_sipg_metric_diag<double>(int, const MetricGeom<double>&, double*, hipStream_t);
template dgmf_status launch_sipg_metric_diag<float>(int, const MetricGeom<double>&, float*, hipStream_t);

dgmf_status launch_metric_fill(int n, const MetricGeom<double>& g, const double* const x0[3], const double* const h[3],
                               const double shinv[9], double shdet, const double* wq, double* cm, double* fm,
                               double* ftau, double* lm, double* ltau, hipStream_t s) {
  FillArgs a{};
  a.g = g;
  for (int d = 0; d < 3; ++d) {
    a.x0[d] = x0[d];
    a.h[d] = h[d];
  }
  for (int i = 0; i < 9; ++i) a.shinv[i] = shinv[i];
  a.shdet = shdet;
  a.k1sq = static_cast<double>(n) * n;
  a.wq = wq;
  const int64_t ncells = static_cast<int64_t>(g.nx) * g.ny * g.nz;
#define X(q)                                                                                               \
  if (n == q) {                                                                                            \
    const unsigned b1 = static_cast<unsigned>((ncells * q * q * q + 255) / 256);                          \
    hipLaunchKernelGGL((k_metric_fill_cells<q>), dim3(b1), dim3(256), 0, s, a, cm);                       \
    DGMF_LAUNCH_CHECK("k_metric_fill_cells");                                                             \
    const unsigned b2 = static_cast<unsigned>((ncells * 6 * q * q + 255) / 256);                          \
    hipLaunchKernelGGL((k_metric_fill_faces<q>), dim3(b2), dim3(256), 0, s, a, fm, ftau, lm, ltau);       \
    DGMF_LAUNCH_CHECK("k_metric_fill_faces");                                                             \
    return DGMF_OK;                                                                                        \
  }
  DGMF_MET_CASES(X)
#undef X
  return fail(DGMF_UNSUPPORTED, "metric fill: degree %d not built", n - 1);
}

dgmf_status launch_metric_fill_curved(int n, const MetricGeom<double>& g, const double* const x0[3],
                                      const double* const h[3], const double lo[3], const double len[3], double amp,
                                      const double* ctab, double* taue, double* cm, double* fm, double* ftau,
                                      double* lm, double* ltau, hipStream_t s) {
  CurvArgs a{};
  a.g = g;
  for (int d = 0; d < 3; ++d) {
    a.map.x0[d] = x0[d];
    a.map.h[d] = h[d];
    a.map.lo[d] = lo[d];
    a.map.len[d] = len[d];
  }
  a.map.amp = amp;
  a.map.nodes = ctab;
  a.k1sq = static_cast<double>(n) * n;
  a.ctab = ctab;
  a.taue = taue;
  const int64_t ncells = static_cast<int64_t>(g.nx) * g.ny * g.nz;
#define X(q)                                                                                               \
  if (n == q) {                                                                                            \
    const unsigned b0 = static_cast<unsigned>((ncells + 255) / 256);                                      \
    hipLaunchKernelGGL((k_curved_tau<q>), dim3(b0), dim3(256), 0, s, a, taue);                            \
    DGMF_LAUNCH_CHECK("k_curved_tau");                                                                    \
    const unsigned b1 = static_cast<unsigned>((ncells * q * q * q + 255) / 256);                          \
    hipLaunchKernelGGL((k_curved_fill_cells<q>), dim3(b1), dim3(256), 0, s, a, cm);                       \
    DGMF_LAUNCH_CHECK("k_curved_fill_cells");                                                             \
    const unsigned b2 = static_cast<unsigned>((ncells * 6 * q * q + 255) / 256);                          \
    hipLaunchKernelGGL((k_curved_fill_faces<q>), dim3(b2), dim3(256), 0, s, a, fm, ftau, lm, ltau);       \
    DGMF_LAUNCH_CHECK("k_curved_fill_faces");                                                             \
    return DGMF_OK;                                                                                        \
  }
  DGMF_MET_CASES(X)
#undef X
  return fail(DGMF_UNSUPPORTED, "metric fill: degree %d not built", n - 1);
}

}  // namespace dgmf
