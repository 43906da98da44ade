// Coupling part of the viscous operator in the symmetric-gradient form
// (Sec. 3.2, implicit viscous step with s = 1, F^nu(u) = 2 nu eps(u)) on
// axis-aligned box meshes (gfx950, fp64).
//
// Writing 2 eps(u) : eps(v) = grad u_c . grad v_c + d_c u_c' d_c' v_c (sums over
// c, c'), the SIPG form splits into the scalar SIPG Helmholtz operator applied
// to every component (mass, Laplacian, penalty tau nu) and nu C(u) with
//   (C u)_{c,i} = sum_c' (d_c' phi_i, d_c u_c')_K
//     - sum_F ( {{d_c u_d}} sigma, phi_i )_F                  (every c; F normal to d)
//     - sum_F ( d_c' phi_i sigma, [u_c'] )_F / 2              (c = d only)
// on a face of direction d with outward normal sigma e_d, [u] the own trace
// minus the neighbour's; on Dirichlet faces (g_u = 0) the average is the own
// value and the second face term has weight 1 instead of 1/2; homogeneous
// Neumann faces add nothing.
//
// 64/n^2 cells per wavefront.  Cell term: per output component c and input
// component c' the tensor product of Kh along c when c' = c, else Ch along c'
// and Ch^T along c, Mh along the rest; the nine products share their x sweeps
// (6 distinct) and their z sweeps (accumulated per line), 21 sweeps in all, run
// in place in six N^3 arrays.  Faces: GLL end points make traces node planes;
// tangential derivatives of a trace use the nodal derivative matrix, the
// normal derivative of u_d the end-point derivatives l_j'(0), l_j'(1) along
// the line (read straight from the field, own and neighbour), and face
// integrals of trace polynomials area (Mh (x) Mh); the six plane integrals of
// a face run as one batch of sweeps along each plane axis.
#include "internal.h"

namespace dgmf {
namespace {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// plane helpers: a face plane is [p2][p1], p1 along t1 (the lower tangential axis), p2 along t2
template <int N>
__device__ __forceinline__ int plane_node(int d, int e, int p1, int p2) {
  if (d == 0) return (p2 * N + p1) * N + e;
  if (d == 1) return (p2 * N + e) * N + p1;
  return (e * N + p2) * N + p1;
}

// Packing: 64/N^2 cells per wavefront, N^2 lanes per cell; lane t of a cell owns
// one line of its cell in every tensor sweep and one node of every face plane.
// Per cell the LDS slice holds six N^3 arrays S0..S5 (the cell-term stages in
// place, S0..S2 ending as the accumulated output of components 0..2) and the
// face planes J (3), A (1), G (3), X (6), which reuse S3..S5 when they fit.
template <int N>
struct EPack {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int TABN = 7 * N2 + 4 * N;
  static constexpr int CPW = 64 / N2 > 0 ? 64 / N2 : 1;
  static constexpr int FACE = 13 * N2;
  static constexpr int SLICE = 6 * N3 + (FACE > 3 * N3 ? FACE - 3 * N3 : 0);
  static constexpr int BYTES = CPW * SLICE * 8;    // per wavefront
  // wavefronts per workgroup: the most resident wavefronts per compute unit
  // (160 KiB of LDS, allocated in 1 KiB steps), fewer per workgroup on ties
  static constexpr int lds_round(int b) { return (b + 1023) / 1024 * 1024; }
  static constexpr int per_cu(int w) { return w * (163840 / lds_round(w * BYTES + TABN * 8)); }
  static constexpr int WAVES = per_cu(1) >= per_cu(2) && per_cu(1) >= per_cu(4) ? 1 : (per_cu(2) >= per_cu(4) ? 2 : 4);
  // register budget for n <= 5: as many wavefronts per SIMD as the LDS admits,
  // at most 3 (larger n would spill)
  static constexpr int MINW = N > 5 || per_cu(WAVES) / 4 < 1 ? 1 : (per_cu(WAVES) / 4 > 3 ? 3 : per_cu(WAVES) / 4);
};

// Compiler-only ordering point (no instruction): keeps the scheduler from
// interleaving consecutive line products, which bounds the live registers.
__device__ __forceinline__ void cfence() { asm volatile("" ::: "memory"); }

// base node and stride of line t along `axis` of an N^3 array
template <int N>
__device__ __forceinline__ void line_of(int axis, int t, int& base, int& stride) {
  constexpr int N2 = N * N;
  const int a = t % N, b = t / N;
  stride = axis == 0 ? 1 : (axis == 1 ? N : N2);
  base = axis == 0 ? (b * N + a) * N : (axis == 1 ? b * N2 + a : b * N + a);
}

template <int N>
__device__ __forceinline__ void load_line(const double* in, int base, int stride, double (&v)[N]) {
#pragma unroll
  for (int m = 0; m < N; ++m) v[m] = in[base + m * stride];
}

template <int N>
__device__ __forceinline__ void store_line(double* out, int base, int stride, const double (&r)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) out[base + i * stride] = r[i];
}

// Tables read with indices uniform over the wavefront: for n <= 5 through the
// constant address space (scalar loads into SGPRs, which the FMAs take
// directly); larger tables would overflow the scalar registers and stay in LDS.
using cdptr = const __attribute__((address_space(4))) double*;
template <bool C>
struct TabPtr {
  using type = const double*;
};
template <>
struct TabPtr<true> {
  using type = cdptr;
};
template <bool C>
__device__ __forceinline__ typename TabPtr<C>::type tab_ptr(const double* global, const double* lds) {
  if constexpr (C) return (cdptr)global;
  else return lds;
}

// r (=, or += when ACC) s M v on one line; M row-major [out][in], transposed when TR
template <int N, bool TR, bool ACC, typename PT>
__device__ __forceinline__ void lmul(PT M, const double (&v)[N], double s, double (&r)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) {
    double a = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) a = fma(TR ? M[m * N + i] : M[i * N + m], v[m], a);
    r[i] = ACC ? fma(s, a, r[i]) : s * a;
  }
}

template <int N, int WAVES>
__global__ void __launch_bounds__(64 * WAVES, EPack<N>::MINW) k_eps_coupling(const double* __restrict__ u,
                                                             double* __restrict__ out,
                                                             const CartGeom<double> g,
                                                             const double* __restrict__ tab, double nu,
                                                             int64_t ncells) {
  using P = EPack<N>;
  constexpr int N2 = P::N2, N3 = P::N3, CPW = P::CPW, SLICE = P::SLICE;
  __shared__ double s_tab[P::TABN];
  __shared__ double s_all[WAVES * CPW * SLICE];
  for (int e = threadIdx.x; e < P::TABN; e += blockDim.x) s_tab[e] = tab[e];
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t first = (static_cast<int64_t>(blockIdx.x) * WAVES + wave) * CPW;
  if (first >= ncells) return;
  const int slot = lane / N2, t = lane % N2;
  const bool act = slot < CPW && first + slot < ncells;
  const int64_t cell = act ? first + slot : first;
  const V3Tab L{N};
  const double* Mh = s_tab + L.Mh();
  const double* Ch = s_tab + L.Ch();
  const double* Dn = s_tab + L.Dn();
  const auto cMh = tab_ptr<(N <= 5)>(tab + L.Mh(), Mh);
  const auto cCh = tab_ptr<(N <= 5)>(tab + L.Ch(), Ch);
  const auto cKh = tab_ptr<(N <= 5)>(tab + L.Kh(), s_tab + L.Kh());
  const double* g0 = s_tab + L.g0();
  const double* g1 = s_tab + L.g1();
  double* S0 = s_all + (wave * CPW + (slot < CPW ? slot : 0)) * SLICE;
  double* S1 = S0 + N3;
  double* S2 = S1 + N3;
  double* S3 = S2 + N3;
  double* S4 = S3 + N3;
  double* S5 = S4 + N3;
  double* J = S3;              // 3 planes: jumps of u_c (indexed by c)
  double* A = J + 3 * N2;      // averaged trace of u_d
  double* G = A + N2;          // 3 planes: averaged d_c u_d (indexed by c)
  double* X = G + 3 * N2;      // 6 planes after the p1 sweeps
  const int64_t Nd = ncells * N3;
  int ci[3];
  ci[0] = static_cast<int>(cell % g.nx);
  ci[1] = static_cast<int>((cell / g.nx) % g.ny);
  ci[2] = static_cast<int>(cell / (static_cast<int64_t>(g.nx) * g.ny));
  double h[3], hi[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    h[d] = g.h[d][ci[d]];
    hi[d] = g.hinv[d][ci[d]];
  }
  const double vol = h[0] * h[1] * h[2];
  double sc[3][3];
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int cp = 0; cp < 3; ++cp) sc[c][cp] = vol * hi[c] * hi[cp];
  // u_0, u_1, u_2 into S0, S2, S5 (the slots their first in-place sweep keeps)
  if (act)
#pragma unroll
    for (int r = 0; r < N; ++r) {
      const int e = t + N2 * r;
      S0[e] = u[cell * N3 + e];
      S2[e] = u[Nd + cell * N3 + e];
      S5[e] = u[2 * Nd + cell * N3 + e];
    }
  wave_sync();
  // ---- cell term O_c = sum_c' s_cc' (op_x op_y op_z) u_c', op along an axis a:
  // Kh if a = c = c', Ch if a = c' != c, Ch^T if a = c != c', else Mh.
  // x: S0 = Kh u0, S1 = Ch u0, S2 = Mh u1, S3 = Ch^T u1, S4 = Ch^T u2, S5 = Mh u2
  if (act) {
    int b, st;
    line_of<N>(0, t, b, st);
    double v[N], r[N];
    load_line<N>(S0, b, st, v);
    lmul<N, false, false>(cKh, v, 1.0, r);
    store_line<N>(S0, b, st, r);
    cfence();
    lmul<N, false, false>(cCh, v, 1.0, r);
    store_line<N>(S1, b, st, r);
    cfence();
    load_line<N>(S2, b, st, v);
    lmul<N, false, false>(cMh, v, 1.0, r);
    store_line<N>(S2, b, st, r);
    cfence();
    lmul<N, true, false>(cCh, v, 1.0, r);
    store_line<N>(S3, b, st, r);
    cfence();
    load_line<N>(S5, b, st, v);
    lmul<N, false, false>(cMh, v, 1.0, r);
    store_line<N>(S5, b, st, r);
    cfence();
    lmul<N, true, false>(cCh, v, 1.0, r);
    store_line<N>(S4, b, st, r);
    cfence();
  }
  wave_sync();
  // y: S0 = s00 Mh S0 + s01 Ch S3 (then Mh along z), S4 = s02 Mh S4 (then Ch),
  //    S1 = s10 Ch^T S1 + s11 Kh S2 (then Mh), S2 = s20 Mh S1 + s21 Ch S2 (then Ch^T),
  //    S5 = s12 Ch^T S5 (then Ch), S3 = s22 Mh S5 (then Kh)
  if (act) {
    int b, st;
    line_of<N>(1, t, b, st);
    double v[N], w[N], r[N];
    load_line<N>(S0, b, st, v);
    load_line<N>(S3, b, st, w);
    lmul<N, false, false>(cMh, v, sc[0][0], r);
    lmul<N, false, true>(cCh, w, sc[0][1], r);
    store_line<N>(S0, b, st, r);
    cfence();
    load_line<N>(S4, b, st, v);
    lmul<N, false, false>(cMh, v, sc[0][2], r);
    store_line<N>(S4, b, st, r);
    cfence();
    load_line<N>(S1, b, st, v);
    load_line<N>(S2, b, st, w);
    lmul<N, true, false>(cCh, v, sc[1][0], r);
    lmul<N, false, true>(cKh, w, sc[1][1], r);
    store_line<N>(S1, b, st, r);
    cfence();
    lmul<N, false, false>(cMh, v, sc[2][0], r);
    lmul<N, false, true>(cCh, w, sc[2][1], r);
    store_line<N>(S2, b, st, r);
    cfence();
    load_line<N>(S5, b, st, v);
    lmul<N, true, false>(cCh, v, sc[1][2], r);
    store_line<N>(S5, b, st, r);
    cfence();
    lmul<N, false, false>(cMh, v, sc[2][2], r);
    store_line<N>(S3, b, st, r);
    cfence();
  }
  wave_sync();
  // z: O0 = Mh S0 + Ch S4 -> S0, O1 = Mh S1 + Ch S5 -> S1, O2 = Ch^T S2 + Kh S3 -> S2
  if (act) {
    int b, st;
    line_of<N>(2, t, b, st);
    double v[N], w[N], r[N];
    load_line<N>(S0, b, st, v);
    load_line<N>(S4, b, st, w);
    lmul<N, false, false>(cMh, v, 1.0, r);
    lmul<N, false, true>(cCh, w, 1.0, r);
    store_line<N>(S0, b, st, r);
    cfence();
    load_line<N>(S1, b, st, v);
    load_line<N>(S5, b, st, w);
    lmul<N, false, false>(cMh, v, 1.0, r);
    lmul<N, false, true>(cCh, w, 1.0, r);
    store_line<N>(S1, b, st, r);
    cfence();
    load_line<N>(S2, b, st, v);
    load_line<N>(S3, b, st, w);
    lmul<N, true, false>(cCh, v, 1.0, r);
    lmul<N, false, true>(cKh, w, 1.0, r);
    store_line<N>(S2, b, st, r);
    cfence();
  }
  wave_sync();
  // ---- faces; this lane's plane node (p1, p2)
  const int p1 = t % N, p2 = t / N;
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const double area = h[t1] * h[t2];
    for (int sd = 0; sd < 2; ++sd) {
      const double sigma = sd ? 1.0 : -1.0;
      const int e = sd ? N - 1 : 0;
      const double* gend = sd ? g1 : g0;      // own end-point derivative row
      const double* gopp = sd ? g0 : g1;      // the neighbour's (its opposite end)
      const int nd = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
      int cc = ci[d] + (sd ? 1 : -1);
      bool interior = true;
      if (cc < 0 || cc >= nd) {
        if (!g.per[d]) interior = false;
        cc = cc < 0 ? nd - 1 : 0;
      }
      const int64_t stride = d == 0 ? 1 : (d == 1 ? g.nx : static_cast<int64_t>(g.nx) * g.ny);
      const int64_t nb = cell + static_cast<int64_t>(cc - ci[d]) * stride;
      const double hinb = interior ? g.hinv[d][cc] : 0.0;
      if (act) {
        // jumps of the three components, averaged trace and normal derivative of u_d
        const double* ud = u + d * Nd;
        double dn_own = 0, dn_nb = 0, ownd = 0, nbd = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          const double o = ud[cell * N3 + plane_node<N>(d, j, p1, p2)];
          dn_own = fma(gend[j], o, dn_own);
          if (j == e) ownd = o;
          if (interior) {
            const double q = ud[nb * N3 + plane_node<N>(d, j, p1, p2)];
            dn_nb = fma(gopp[j], q, dn_nb);
            if (j == N - 1 - e) nbd = q;
          }
        }
        const int q = p2 * N + p1;
        J[d * N2 + q] = ownd - nbd;
        A[q] = interior ? 0.5 * (ownd + nbd) : ownd;
        G[d * N2 + q] = interior ? 0.5 * (hi[d] * dn_own + hinb * dn_nb) : hi[d] * dn_own;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int tk = k == 0 ? t1 : t2;
          const double own = u[tk * Nd + cell * N3 + plane_node<N>(d, e, p1, p2)];
          const double oth = interior ? u[tk * Nd + nb * N3 + plane_node<N>(d, N - 1 - e, p1, p2)] : 0.0;
          J[tk * N2 + q] = own - oth;
        }
      }
      wave_sync();
      // tangential derivatives of the averaged trace: G_t1 = hinv_t1 Dn_p1 A, G_t2 = hinv_t2 Dn_p2 A
      if (act) {
        double r1 = 0, r2 = 0;
#pragma unroll
        for (int m = 0; m < N; ++m) {
          r1 = fma(Dn[p1 * N + m], A[p2 * N + m], r1);
          r2 = fma(Dn[p2 * N + m], A[m * N + p1], r2);
        }
        G[t1 * N2 + t] = hi[t1] * r1;
        G[t2 * N2 + t] = hi[t2] * r2;
      }
      wave_sync();
      // six plane integrals, first along p1:
      //   0..2: (Mh (x) Mh) G_c      3: (Ch_p1, Mh_p2) J_t1      4: (Mh_p1, Ch_p2) J_t2      5: (Mh (x) Mh) J_d
      if (act) {
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const double* in = k < 3 ? G + k * N2 : J + (k == 3 ? t1 : (k == 4 ? t2 : d)) * N2;
          const double* M = k == 3 ? Ch : Mh;
          double r = 0;
#pragma unroll
          for (int m = 0; m < N; ++m) r = fma(M[p1 * N + m], in[p2 * N + m], r);
          X[k * N2 + t] = r;
        }
      }
      wave_sync();
      if (act) {
        double Y[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) {
          const double* M = k == 4 ? Ch : Mh;
          double r = 0;
#pragma unroll
          for (int m = 0; m < N; ++m) r = fma(M[p2 * N + m], X[k * N2 + m * N + p1], r);
          Y[k] = r;
        }
        // term 2 on the plane of every component; term 1 on component d (plane: the
        // tangential test derivatives; the whole normal line: the test normal derivative)
        // a Neumann side adds nothing (U* = u_h there; the flux F^nu* is data)
        const double sa = (interior || !((g.neu >> (2 * d + sd)) & 1)) ? sigma * area : 0.0;
        const double w1 = (interior ? 0.5 : 1.0) * sa;
        const double Yd = d == 0 ? Y[0] : (d == 1 ? Y[1] : Y[2]);
        const double Yt1 = t1 == 0 ? Y[0] : Y[1];
        const double Yt2 = t2 == 1 ? Y[1] : Y[2];
        double* Od = S0 + d * N3;
#pragma unroll
        for (int id = 0; id < N; ++id) {
          double v = w1 * hi[d] * gend[id] * Y[5];
          if (id == e) v += sa * Yd + w1 * (hi[t1] * Y[3] + hi[t2] * Y[4]);
          Od[plane_node<N>(d, id, p1, p2)] -= v;
        }
        S0[t1 * N3 + plane_node<N>(d, e, p1, p2)] -= sa * Yt1;
        S0[t2 * N3 + plane_node<N>(d, e, p1, p2)] -= sa * Yt2;
      }
      wave_sync();
    }
  }
  if (act)
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int r = 0; r < N; ++r) {
        const int e = t + N2 * r;
        const int64_t at = c * Nd + cell * N3 + e;
        out[at] = fma(nu, S0[c * N3 + e], out[at]);
      }
}

template <int N>
dgmf_status eps_n(const CartGeom<double>& g, const double* tab, const double* u, double* out, double nu,
                  int64_t ncells, hipStream_t s) {
  constexpr int W = EPack<N>::WAVES, CPW = EPack<N>::CPW;
  const int64_t waves = (ncells + CPW - 1) / CPW;
  const int64_t blocks = (waves + W - 1) / W;
  if (blocks > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "viscous: too many cells for one launch");
  hipLaunchKernelGGL((k_eps_coupling<N, W>), dim3(static_cast<unsigned>(blocks)), dim3(64 * W), 0, s, u, out, g,
                     tab, nu, ncells);
  DGMF_LAUNCH_CHECK("k_eps_coupling");
  return DGMF_OK;
}

}  // namespace

dgmf_status launch_eps_coupling(int n, const CartGeom<double>& g, const double* tab, const double* u, double* out,
                                double nu, int64_t ncells, hipStream_t s) {
  switch (n) {
    case 2: return eps_n<2>(g, tab, u, out, nu, ncells, s);
    case 3: return eps_n<3>(g, tab, u, out, nu, ncells, s);
    case 4: return eps_n<4>(g, tab, u, out, nu, ncells, s);
    case 5: return eps_n<5>(g, tab, u, out, nu, ncells, s);
    case 6: return eps_n<6>(g, tab, u, out, nu, ncells, s);
    case 7: return eps_n<7>(g, tab, u, out, nu, ncells, s);
    case 8: return eps_n<8>(g, tab, u, out, nu, ncells, s);
    default: return fail(DGMF_UNSUPPORTED, "viscous: n = %d not built", n);
  }
}

}  // namespace dgmf
