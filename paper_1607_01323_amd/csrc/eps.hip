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
// minus the neighbour's; on boundary faces (g_u = 0) the average is the own
// value and the second face term has weight 1 instead of 1/2.
//
// One cell per wavefront.  Cell term: 27 tensor sweeps (per output component
// c and input component c': Kh along c when c' = c, else Ch along c' and Ch^T
// along c, Mh along the rest).  Faces: GLL end points make traces node planes;
// tangential derivatives of a trace use the nodal derivative matrix, the
// normal derivative of u_d the end-point derivatives l_j'(0), l_j'(1) along
// the line, and face integrals of trace polynomials area (Mh (x) Mh); the six
// plane integrals of a face run as one batch of sweeps along each plane axis,
// so a face costs six wavefront steps.
#include "internal.h"

namespace dgmf {
namespace {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// out (=, or += when ACC) scale * (M along axis) in, M row-major [out][in] (TR: transposed)
template <int N, bool TR, bool ACC>
__device__ __forceinline__ void sweep(const double* M, int axis, const double* in, double* out, double scale,
                                      int lane) {
  constexpr int N2 = N * N;
  const int stride = axis == 0 ? 1 : (axis == 1 ? N : N2);
  for (int L = lane; L < N2; L += 64) {
    const int a = L % N, b = L / N;
    const int base = axis == 0 ? (b * N + a) * N : (axis == 1 ? b * N2 + a : b * N + a);
    double v[N];
#pragma unroll
    for (int m = 0; m < N; ++m) v[m] = in[base + m * stride];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double r = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) r = fma(TR ? M[m * N + i] : M[i * N + m], v[m], r);
      if (ACC) out[base + i * stride] += scale * r;
      else out[base + i * stride] = scale * r;
    }
  }
}

// plane helpers: a face plane is [p2][p1], p1 along t1 (the lower tangential axis), p2 along t2
template <int N>
__device__ __forceinline__ int plane_node(int d, int e, int p1, int p2) {
  if (d == 0) return (p2 * N + p1) * N + e;
  if (d == 1) return (p2 * N + e) * N + p1;
  return (e * N + p2) * N + p1;
}

template <int N>
struct EShape {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int TABN = 7 * N2 + 4 * N;
  // U (3 N3), O (3 N3), T1, T2, NB (N3 each), planes: NBt (2), J (3), G (3), A (1), X (6), Y (6)
  static constexpr int SLICE = 9 * N3 + 21 * N2;
  static constexpr int BYTES = SLICE * 8;
  // wavefronts per workgroup: the most resident wavefronts per compute unit
  // (160 KiB of LDS, allocated in 1 KiB steps), fewer per workgroup on ties
  static constexpr int lds_round(int b) { return (b + 1023) / 1024 * 1024; }
  static constexpr int per_cu(int w) { return w * (163840 / lds_round(w * BYTES + TABN * 8)); }
  static constexpr int WAVES = per_cu(1) >= per_cu(2) && per_cu(1) >= per_cu(4) ? 1 : (per_cu(2) >= per_cu(4) ? 2 : 4);
};

template <int N>
__global__ void __launch_bounds__(64 * EShape<N>::WAVES) k_eps_coupling(const double* __restrict__ u,
                                                                        double* __restrict__ out,
                                                                        const CartGeom<double> g,
                                                                        const double* __restrict__ tab, double nu,
                                                                        int64_t ncells) {
  using SH = EShape<N>;
  constexpr int N2 = SH::N2, N3 = SH::N3;
  __shared__ double s_tab[SH::TABN];
  __shared__ double s_all[SH::WAVES * SH::SLICE];
  for (int e = threadIdx.x; e < SH::TABN; e += blockDim.x) s_tab[e] = tab[e];
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t cell = static_cast<int64_t>(blockIdx.x) * SH::WAVES + wave;
  if (cell >= ncells) return;
  const V3Tab L{N};
  const double* Mh = s_tab + L.Mh();
  const double* Ch = s_tab + L.Ch();
  const double* Kh = s_tab + L.Kh();
  const double* Dn = s_tab + L.Dn();
  const double* g0 = s_tab + L.g0();
  const double* g1 = s_tab + L.g1();
  double* U = s_all + wave * SH::SLICE;
  double* O = U + 3 * N3;
  double* T1 = O + 3 * N3;
  double* T2 = T1 + N3;
  double* NB = T2 + N3;
  double* NBt = NB + N3;       // 2 planes: the neighbour's other two components
  double* J = NBt + 2 * N2;    // 3 planes: jumps of u_c'
  double* G = J + 3 * N2;      // 3 planes: averaged d_c u_d
  double* A = G + 3 * N2;      // averaged trace of u_d
  double* X = A + N2;          // 6 planes after the p1 sweeps
  double* Y = X + 6 * N2;      // 6 planes after the p2 sweeps
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
  for (int e = lane; e < 3 * N3; e += 64) {
    U[e] = u[(e / N3) * Nd + cell * N3 + e % N3];
    O[e] = 0.0;
  }
  wave_sync();
  // ---- cell term: O_c += sum_c' s_cc' (op along x, y, z) u_c'
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int cp = 0; cp < 3; ++cp) {
      const double* M3[3];
      bool tr[3] = {false, false, false};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) M3[ax] = Mh;
      if (cp == c) {
        M3[c] = Kh;
      } else {
        M3[cp] = Ch;        // test derivative along c'
        M3[c] = Ch;         // trial derivative along c: Ch^T
        tr[c] = true;
      }
      const double sc = vol * hi[c] * hi[cp];
      if (tr[0]) sweep<N, true, false>(M3[0], 0, U + cp * N3, T1, 1.0, lane);
      else sweep<N, false, false>(M3[0], 0, U + cp * N3, T1, 1.0, lane);
      wave_sync();
      if (tr[1]) sweep<N, true, false>(M3[1], 1, T1, T2, 1.0, lane);
      else sweep<N, false, false>(M3[1], 1, T1, T2, 1.0, lane);
      wave_sync();
      if (tr[2]) sweep<N, true, true>(M3[2], 2, T2, O + c * N3, sc, lane);
      else sweep<N, false, true>(M3[2], 2, T2, O + c * N3, sc, lane);
      wave_sync();
    }
  // ---- faces
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const double area = h[t1] * h[t2];
    for (int sd = 0; sd < 2; ++sd) {
      const double sigma = sd ? 1.0 : -1.0;
      const int e = sd ? N - 1 : 0;
      const double* gend = sd ? g1 : g0;      // own end-point derivative row
      const double* gopp = sd ? g0 : g1;      // the neighbour's (its opposite end)
      // neighbour across the face
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
      if (interior) {
        for (int q = lane; q < N3; q += 64) NB[q] = u[d * Nd + nb * N3 + q];
        for (int q = lane; q < 2 * N2; q += 64) {
          const int k = q / N2, r = q % N2;
          NBt[q] = u[(k == 0 ? t1 : t2) * Nd + nb * N3 + plane_node<N>(d, N - 1 - e, r % N, r / N)];
        }
      }
      wave_sync();
      for (int q = lane; q < N2; q += 64) {
        const int p1 = q % N, p2 = q / N;
        // jumps of the three components, averaged trace of u_d, averaged normal derivative of u_d
        const double ownd = U[d * N3 + plane_node<N>(d, e, p1, p2)];
        const double nbd = interior ? NB[plane_node<N>(d, N - 1 - e, p1, p2)] : 0.0;
        J[d * N2 + q] = ownd - nbd;
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int tk = k == 0 ? t1 : t2;
          const double own = U[tk * N3 + plane_node<N>(d, e, p1, p2)];
          J[tk * N2 + q] = own - (interior ? NBt[k * N2 + q] : 0.0);
        }
        A[q] = interior ? 0.5 * (ownd + nbd) : ownd;
        double dn_own = 0, dn_nb = 0;
#pragma unroll
        for (int j = 0; j < N; ++j) {
          dn_own = fma(gend[j], U[d * N3 + plane_node<N>(d, j, p1, p2)], dn_own);
          if (interior) dn_nb = fma(gopp[j], NB[plane_node<N>(d, j, p1, p2)], dn_nb);
        }
        G[d * N2 + q] = interior ? 0.5 * (hi[d] * dn_own + hinb * dn_nb) : hi[d] * dn_own;
      }
      wave_sync();
      // tangential derivatives of the averaged trace, scaled: G_t1 = hinv_t1 Dn_p1 A, G_t2 = hinv_t2 Dn_p2 A
      for (int w = lane; w < 2 * N2; w += 64) {
        const int k = w / N2, q = w % N2, p1 = q % N, p2 = q / N;
        double r = 0;
#pragma unroll
        for (int m = 0; m < N; ++m)
          r = fma(k == 0 ? Dn[p1 * N + m] : Dn[p2 * N + m], k == 0 ? A[p2 * N + m] : A[m * N + p1], r);
        G[(k == 0 ? t1 : t2) * N2 + q] = (k == 0 ? hi[t1] : hi[t2]) * r;
      }
      wave_sync();
      // six plane integrals at once, first along p1 then along p2:
      //   0..2: (Mh (x) Mh) G_c      3: (Ch_p1, Mh_p2) J_t1      4: (Mh_p1, Ch_p2) J_t2      5: (Mh (x) Mh) J_d
      for (int w = lane; w < 6 * N2; w += 64) {
        const int k = w / N2, q = w % N2, p1 = q % N, p2 = q / N;
        const double* in = k < 3 ? G + k * N2 : J + (k == 3 ? t1 : (k == 4 ? t2 : d)) * N2;
        const double* M = k == 3 ? Ch : Mh;
        double r = 0;
#pragma unroll
        for (int m = 0; m < N; ++m) r = fma(M[p1 * N + m], in[p2 * N + m], r);
        X[w] = r;
      }
      wave_sync();
      for (int w = lane; w < 6 * N2; w += 64) {
        const int k = w / N2, q = w % N2, p1 = q % N, p2 = q / N;
        const double* M = k == 4 ? Ch : Mh;
        double r = 0;
#pragma unroll
        for (int m = 0; m < N; ++m) r = fma(M[p2 * N + m], X[k * N2 + m * N + p1], r);
        Y[w] = r;
      }
      wave_sync();
      // accumulate: term 2 on the plane of every component, term 1 on component d (plane: tangential
      // test derivatives; every node along the normal: the test function's normal derivative)
      const double w1 = (interior ? 0.5 : 1.0) * sigma * area;
      for (int w = lane; w < N3 + 2 * N2; w += 64) {
        if (w < N3) {
          int id, p1, p2;
          if (d == 0) { id = w % N; p1 = (w / N) % N; p2 = w / N2; }
          else if (d == 1) { id = (w / N) % N; p1 = w % N; p2 = w / N2; }
          else { id = w / N2; p1 = w % N; p2 = (w / N) % N; }
          const int q = p2 * N + p1;
          double v = w1 * hi[d] * gend[id] * Y[5 * N2 + q];
          if (id == e) v += sigma * area * Y[d * N2 + q] + w1 * (hi[t1] * Y[3 * N2 + q] + hi[t2] * Y[4 * N2 + q]);
          O[d * N3 + w] -= v;
        } else {
          const int k = (w - N3) / N2, q = (w - N3) % N2;
          const int c = k == 0 ? t1 : t2;
          O[c * N3 + plane_node<N>(d, e, q % N, q / N)] -= sigma * area * Y[c * N2 + q];
        }
      }
      wave_sync();
    }
  }
  for (int e = lane; e < 3 * N3; e += 64) {
    const int64_t at = (e / N3) * Nd + cell * N3 + e % N3;
    out[at] = fma(nu, O[e], out[at]);
  }
}

template <int N>
dgmf_status eps_n(const CartGeom<double>& g, const double* tab, const double* u, double* out, double nu,
                  int64_t ncells, hipStream_t s) {
  constexpr int W = EShape<N>::WAVES;
  const int64_t blocks = (ncells + W - 1) / W;
  if (blocks > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "viscous: too many cells for one launch");
  hipLaunchKernelGGL((k_eps_coupling<N>), dim3(static_cast<unsigned>(blocks)), dim3(64 * W), 0, s, u, out, g, tab,
                     nu, ncells);
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
