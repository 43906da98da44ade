// Operators of variant V3c on axis-aligned box meshes (gfx950, fp64).
//
// Divergence A (eq. av3 without gamma_0/dt) and gradient B (eq. bv3 without
// dt/gamma_0), with the central average on interior faces and the cell's own
// trace on boundary faces (the ND extension of Sec. 3.1):
//   (A u)_i = sum_a (d_a phi_i, u_a)_K - (phi_i, {{u}}.n)_dK
//   (B p)_{i,a} = (d_a phi_i, p)_K - (phi_i, {{p}} n_a)_dK
// On an axis-aligned cell with sizes h the cell terms are tensor products of
// the 1D mass Mh and Ch[i][j] = int_0^1 l_i' l_j scaled by |det J| / h_a,
// e.g. (d_x phi, u)_K = (hy hz) (Mh (x) Mh (x) Ch) u.  GLL nodes include the
// end points, so a face trace is the node plane on that face and the face
// integral of a trace polynomial is area (Mh (x) Mh) on the plane.
//
// The div-div projection (eq. div-div, eq. project with tau_C = 0) is cell
// local: (M_e + tau_e D_e) u = rhs_e with D_e = (div v, div u)_K.  Each cell is
// solved by its own CG (Sec. 5.1, projection solver: element-local CG
// preconditioned by the inverse mass), one wavefront per cell with every
// vector in the wavefront's LDS slice, iterating until its own residual falls
// below rtol times its own right-hand side; D_e is applied through the Gauss
// points (k+1 per direction): div at the points from S and D sweeps, then the
// transposed sweeps.
//
// Layout: A and B pack 64/n^2 cells per wavefront with one line (and one face
// node) per lane; the projection packs 64/SS cells per wavefront, SS the
// smallest power of two >= n^2.  A few wavefronts per workgroup (LDS bound),
// wavefront barriers only after the tables are staged.
#include "internal.h"

namespace dgmf {
namespace {

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

struct CellIdx {
  int c[3];
  double h[3];
};

__device__ __forceinline__ CellIdx cell_of(const CartGeom<double>& g, int64_t cell) {
  CellIdx r;
  r.c[0] = static_cast<int>(cell % g.nx);
  const int64_t q = cell / g.nx;
  r.c[1] = static_cast<int>(q % g.ny);
  r.c[2] = static_cast<int>(q / g.ny);
#pragma unroll
  for (int d = 0; d < 3; ++d) r.h[d] = g.h[d][r.c[d]];
  return r;
}

// neighbour across face (d, s) or -1 on a boundary face
__device__ __forceinline__ int64_t nb_of(const CartGeom<double>& g, const CellIdx& ci, int64_t cell, int d, int s) {
  const int nd = d == 0 ? g.nx : (d == 1 ? g.ny : g.nz);
  int cc = ci.c[d] + (s ? 1 : -1);
  if (cc < 0 || cc >= nd) {
    if (!g.per[d]) return -1;
    cc = cc < 0 ? nd - 1 : 0;
  }
  const int64_t stride = d == 0 ? 1 : (d == 1 ? g.nx : static_cast<int64_t>(g.nx) * g.ny);
  return cell + static_cast<int64_t>(cc - ci.c[d]) * stride;
}

// node index of entry (p1, p2) of the node plane e along direction d (p1, p2: the
// other two directions in increasing order)
template <int N>
__device__ __forceinline__ int plane_node(int d, int e, int p1, int p2) {
  if (d == 0) return (p2 * N + p1) * N + e;
  if (d == 1) return (p2 * N + e) * N + p1;
  return (e * N + p2) * N + p1;
}

template <int N>
struct V3Shape {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int TABN = 5 * N2 + 2 * N;   // the V3Tab entries these kernels use
};

// Tables read with indices uniform over the wavefront: up to n = NMAX through
// the constant address space (scalar loads into SGPRs, which the FMAs take
// directly); for larger n the kernel's tables would overflow the scalar
// registers (hundreds of spills) and stay in LDS.  NMAX: 7 for the divergence
// and gradient, 6 for the projection, which keeps more tables live.
using cdptr = const __attribute__((address_space(4))) double*;
template <bool C>
struct TabPtr {
  using type = const double*;
};
template <>
struct TabPtr<true> {
  using type = cdptr;
};
template <int N, int NMAX>
__device__ __forceinline__ typename TabPtr<(N <= NMAX)>::type tab_ptr(const double* global, const double* lds) {
  if constexpr (N <= NMAX) return (cdptr)global;
  else return lds;
}

// One line along `axis` of an N^3 array per lane (line t = a + N b), as sweep().
template <int N, bool TR, bool ACC, typename PT>
__device__ __forceinline__ void sweep1(PT M, int axis, const double* in, double* out, double scale, int t) {
  constexpr int N2 = N * N;
  const int stride = axis == 0 ? 1 : (axis == 1 ? N : N2);
  const int a = t % N, b = t / N;
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

// Packing of the divergence and gradient kernels: 64/N^2 cells per
// wavefront, N^2 lanes per cell; lane t of a cell owns one line in every
// sweep and one node of every face plane.  Every sweep runs in place (a lane
// reads its whole line before writing it), so a cell needs only three N^3
// arrays (the gradient two face planes more); SLICE doubles per cell.
template <int N, int SLICE_>
struct XPack {
  static constexpr int N2 = N * N, N3 = N2 * N;
  static constexpr int CPW = 64 / N2 > 0 ? 64 / N2 : 1;
  static constexpr int SLICE = SLICE_;
  static constexpr int BYTES = CPW * SLICE * 8;     // per wavefront
  static constexpr int lds_round(int b) { return (b + 1023) / 1024 * 1024; }
  static constexpr int per_cu(int w) { return w * (163840 / lds_round(w * BYTES + V3Shape<N>::TABN * 8)); }
  static constexpr int WAVES = per_cu(1) >= per_cu(2) && per_cu(1) >= per_cu(4) ? 1 : (per_cu(2) >= per_cu(4) ? 2 : 4);
};
template <int N>
using DivPack = XPack<N, 3 * N * N * N>;
template <int N>
using GradPack = XPack<N, 3 * N * N * N + 2 * N * N>;

// Face term of one face on this lane's plane node: O[plane] -= sigma area (Mh (x) Mh) avg,
// avg = central average of the own plane `own` and the neighbour's (or own on a boundary face).
template <int N>
__device__ __forceinline__ void face_plane_term(const double* Mh, double* F, double* Oc, double own, double other,
                                                bool interior, int d, int e, double sg, int t, bool act) {
  constexpr int N2 = N * N;
  const int p1 = t % N, p2 = t / N;
  if (act) F[t] = interior ? 0.5 * (own + other) : own;
  wave_sync();
  double r = 0;
  if (act) {
#pragma unroll
    for (int m = 0; m < N; ++m) r = fma(Mh[p1 * N + m], F[p2 * N + m], r);
    F[N2 + t] = r;
  }
  wave_sync();
  if (act) {
    r = 0;
#pragma unroll
    for (int m = 0; m < N; ++m) r = fma(Mh[p2 * N + m], F[N2 + m * N + p1], r);
    Oc[plane_node<N>(d, e, p1, p2)] -= sg * r;
  }
  wave_sync();
}

// ------------------------------------------------------------ divergence --
template <int N, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_v3_divergence(const double* __restrict__ u, double* __restrict__ out,
                                                              const CartGeom<double> g,
                                                              const double* __restrict__ tab, int64_t ncells) {
  using X = DivPack<N>;
  constexpr int N2 = X::N2, N3 = X::N3, CPW = X::CPW, SLICE = X::SLICE;
  __shared__ double s_tab[V3Shape<N>::TABN];
  __shared__ double s_all[WAVES * CPW * SLICE];
  for (int e = threadIdx.x; e < V3Shape<N>::TABN; e += blockDim.x) s_tab[e] = tab[e];
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t first = (static_cast<int64_t>(blockIdx.x) * WAVES + wave) * CPW;
  if (first >= ncells) return;
  const int slot = lane / N2, t = lane % N2;
  const bool act = slot < CPW && first + slot < ncells;
  const int64_t cell = act ? first + slot : first;
  const V3Tab L{N};
  const double* Mh = s_tab + L.Mh();
  const auto cMh = tab_ptr<N, 7>(tab + L.Mh(), Mh);
  const auto cCh = tab_ptr<N, 7>(tab + L.Ch(), s_tab + L.Ch());
  double* P0 = s_all + (wave * CPW + (slot < CPW ? slot : 0)) * SLICE;   // u_x, then the output
  double* P1 = P0 + N3;                 // u_y, then the face plane scratch (2 N2)
  double* P2 = P1 + N3;                 // u_z
  const int64_t Nd = ncells * N3;
  const CellIdx ci = cell_of(g, cell);
  const double vol = ci.h[0] * ci.h[1] * ci.h[2];
  double s[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) s[a] = vol / ci.h[a];
  if (act)
#pragma unroll
    for (int r = 0; r < 3 * N; ++r) {
      const int e = t + N2 * r;
      P0[e] = u[(e / N3) * Nd + cell * N3 + e % N3];
    }
  wave_sync();
  if (act) {
    sweep1<N, false, false>(cCh, 0, P0, P0, 1.0, t);                    // Ch_x u_x
    sweep1<N, false, false>(cMh, 0, P1, P1, 1.0, t);                    // Mh_x u_y
    sweep1<N, false, false>(cMh, 0, P2, P2, 1.0, t);                    // Mh_x u_z
  }
  wave_sync();
  if (act) {
    sweep1<N, false, false>(cMh, 1, P0, P0, s[0], t);                   // sx Mh_y Ch_x u_x
    sweep1<N, false, true>(cCh, 1, P1, P0, s[1], t);                    // + sy Ch_y Mh_x u_y (same line)
    sweep1<N, false, false>(cMh, 1, P2, P2, s[2], t);                   // sz Mh_y Mh_x u_z
  }
  wave_sync();
  if (act) {
    sweep1<N, false, false>(cMh, 2, P0, P0, 1.0, t);
    sweep1<N, false, true>(cCh, 2, P2, P0, 1.0, t);                     // same line
  }
  wave_sync();
  // faces: O -= sign area (Mh (x) Mh) {{u_d}} on the face plane
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const double area = ci.h[t1] * ci.h[t2];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int e = sd ? N - 1 : 0;
      const int64_t nb = nb_of(g, ci, cell, d, sd);
      const int p1 = t % N, p2 = t / N;
      const double own = act ? u[d * Nd + cell * N3 + plane_node<N>(d, e, p1, p2)] : 0.0;
      const double other = (act && nb >= 0) ? u[d * Nd + nb * N3 + plane_node<N>(d, N - 1 - e, p1, p2)] : 0.0;
      face_plane_term<N>(Mh, P1, P0, own, other, nb >= 0, d, e, (sd ? 1.0 : -1.0) * area, t, act);
    }
  }
  if (act)
#pragma unroll
    for (int r = 0; r < N; ++r) out[cell * N3 + t + N2 * r] = P0[t + N2 * r];
}

// -------------------------------------------------------------- gradient --
template <int N, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_v3_gradient(const double* __restrict__ p, double* __restrict__ out,
                                                            const CartGeom<double> g, const double* __restrict__ tab,
                                                            int64_t ncells) {
  using X = GradPack<N>;
  constexpr int N2 = X::N2, N3 = X::N3, CPW = X::CPW, SLICE = X::SLICE;
  __shared__ double s_tab[V3Shape<N>::TABN];
  __shared__ double s_all[WAVES * CPW * SLICE];
  for (int e = threadIdx.x; e < V3Shape<N>::TABN; e += blockDim.x) s_tab[e] = tab[e];
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t first = (static_cast<int64_t>(blockIdx.x) * WAVES + wave) * CPW;
  if (first >= ncells) return;
  const int slot = lane / N2, t = lane % N2;
  const bool act = slot < CPW && first + slot < ncells;
  const int64_t cell = act ? first + slot : first;
  const V3Tab L{N};
  const double* Mh = s_tab + L.Mh();
  const auto cMh = tab_ptr<N, 7>(tab + L.Mh(), Mh);
  const auto cCh = tab_ptr<N, 7>(tab + L.Ch(), s_tab + L.Ch());
  double* O3 = s_all + (wave * CPW + (slot < CPW ? slot : 0)) * SLICE;  // 3 N3: output components
  double* P = O3 + 2 * N3;              // p, in the slot of output component 2
  double* F = O3 + 3 * N3;              // 2 N2: face plane scratch
  const int64_t Nd = ncells * N3;
  const CellIdx ci = cell_of(g, cell);
  const double vol = ci.h[0] * ci.h[1] * ci.h[2];
  double s[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) s[a] = vol / ci.h[a];
  if (act)
#pragma unroll
    for (int r = 0; r < N; ++r) P[t + N2 * r] = p[cell * N3 + t + N2 * r];
  wave_sync();
  if (act) {
    sweep1<N, false, false>(cCh, 0, P, O3, 1.0, t);                     // Ch_x p
    sweep1<N, false, false>(cMh, 0, P, P, 1.0, t);                      // Mh_x p (in place, after the read)
  }
  wave_sync();
  if (act) {
    sweep1<N, false, false>(cMh, 1, O3, O3, 1.0, t);                    // Mh_y Ch_x p
    sweep1<N, false, false>(cCh, 1, P, O3 + N3, 1.0, t);                // Ch_y Mh_x p
    sweep1<N, false, false>(cMh, 1, P, P, 1.0, t);                      // Mh_y Mh_x p
  }
  wave_sync();
  if (act) {
    sweep1<N, false, false>(cMh, 2, O3, O3, s[0], t);
    sweep1<N, false, false>(cMh, 2, O3 + N3, O3 + N3, s[1], t);
    sweep1<N, false, false>(cCh, 2, P, P, s[2], t);
  }
  wave_sync();
  // faces: O_d -= sign area (Mh (x) Mh) {{p}} on the face plane
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int t1 = d == 0 ? 1 : 0, t2 = d == 2 ? 1 : 2;
    const double area = ci.h[t1] * ci.h[t2];
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
      const int e = sd ? N - 1 : 0;
      const int64_t nb = nb_of(g, ci, cell, d, sd);
      const int p1 = t % N, p2 = t / N;
      const double own = act ? p[cell * N3 + plane_node<N>(d, e, p1, p2)] : 0.0;
      const double other = (act && nb >= 0) ? p[nb * N3 + plane_node<N>(d, N - 1 - e, p1, p2)] : 0.0;
      face_plane_term<N>(Mh, F, O3 + d * N3, own, other, nb >= 0, d, e, (sd ? 1.0 : -1.0) * area, t, act);
    }
  }
  if (act)
#pragma unroll
    for (int r = 0; r < 3 * N; ++r) {
      const int e = t + N2 * r;
      out[(e / N3) * Nd + cell * N3 + e % N3] = O3[e];
    }
}

// ------------------------------------------------------------------ tau_D --
// tau = zeta |u_bar| V^(1/3) dt, u_bar_a = sum_i gw_i u_a,i (gw: basis integrals on the unit cube)
template <int N>
__global__ void __launch_bounds__(256) k_v3_tau(const double* __restrict__ u, const CartGeom<double> g,
                                                const double* __restrict__ tab, double zeta, double dt,
                                                double* __restrict__ tau, int64_t ncells) {
  constexpr int N2 = N * N, N3 = N2 * N;
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int64_t cell = static_cast<int64_t>(blockIdx.x) * 4 + wave;
  if (cell >= ncells) return;
  const double* gw = tab + V3Tab{N}.gw();
  const int64_t Nd = ncells * N3;
  double a[3] = {0, 0, 0};
  for (int e = lane; e < N3; e += 64) {
    const double w = gw[e % N] * gw[(e / N) % N] * gw[e / N2];
#pragma unroll
    for (int c = 0; c < 3; ++c) a[c] = fma(w, u[c * Nd + cell * N3 + e], a[c]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) a[c] += __shfl_xor(a[c], o, 64);
  if (lane == 0) {
    const CellIdx ci = cell_of(g, cell);
    const double vol = ci.h[0] * ci.h[1] * ci.h[2];
    tau[cell] = zeta * sqrt(a[0] * a[0] + a[1] * a[1] + a[2] * a[2]) * cbrt(vol) * dt;
  }
}

// ------------------------------------------------------ projection (CG) --
// Packing: each cell owns an aligned group of SS lanes (the smallest power of
// two >= N^2, so that a butterfly over the group sums a cell's partials), 64/SS
// cells per wavefront.  Lane t < N^2 of a group owns one line of its cell in
// every sweep and the nodes t + N^2 j (j < 3N) in vector operations, whose x
// it keeps in registers.  Per cell the LDS slice holds r, p, q and one
// 3-component temporary T, which also holds z = M_e^{-1} r between the
// preconditioner and the update of p.
template <int N>
struct PPack {
  static constexpr int N2 = N * N, N3 = N2 * N, V = 3 * N3;
  static constexpr int SS = N2 <= 4 ? 4 : (N2 <= 8 ? 8 : (N2 <= 16 ? 16 : (N2 <= 32 ? 32 : 64)));
  static constexpr int CPW = 64 / SS;
  static constexpr int SLICE = 4 * V;
  static constexpr int BYTES = CPW * SLICE * 8;     // per wavefront
  static constexpr int lds_round(int b) { return (b + 1023) / 1024 * 1024; }
  static constexpr int per_cu(int w) { return w * (163840 / lds_round(w * BYTES + V3Shape<N>::TABN * 8)); }
  static constexpr int WAVES = per_cu(1) >= per_cu(2) && per_cu(1) >= per_cu(4) ? 1 : (per_cu(2) >= per_cu(4) ? 2 : 4);
};

// sum over the aligned group of SS lanes (every lane of the group gets the same value)
template <int SS>
__device__ __forceinline__ double group_sum(double v) {
#pragma unroll
  for (int o = SS / 2; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Compiler-only ordering point (no instruction): keeps the scheduler from
// interleaving consecutive sweeps, which bounds the live registers to one
// sweep's line and matrix entries.
__device__ __forceinline__ void cfence() { asm volatile("" ::: "memory"); }

// q = (M_e (x) I_3 + tau D_e) p on one cell; T: 3-component temporary.  Lane t owns line t.
template <int N>
__device__ __forceinline__ void proj_apply(const double* tg, const double* tb, const double* p, double* q, double* T,
                                           const double (&hinv)[3], double vol, double tau, int t, bool act) {
  constexpr int N3 = N * N * N;
  const V3Tab L{N};
  const auto Mh = tab_ptr<N, 6>(tg + L.Mh(), tb + L.Mh());
  const auto S = tab_ptr<N, 6>(tg + L.S(), tb + L.S());
  const auto D = tab_ptr<N, 6>(tg + L.D(), tb + L.D());
  const double* w = tb + L.w();
  // mass: q_a = vol Mh_z Mh_y Mh_x p_a (the y and z sweeps in place)
  if (act)
#pragma unroll 1
    for (int a = 0; a < 3; ++a) sweep1<N, false, false>(Mh, 0, p + a * N3, q + a * N3, 1.0, t);
  wave_sync();
  if (act)
#pragma unroll 1
    for (int a = 0; a < 3; ++a) sweep1<N, false, false>(Mh, 1, q + a * N3, q + a * N3, 1.0, t);
  wave_sync();
  if (act)
#pragma unroll 1
    for (int a = 0; a < 3; ++a) sweep1<N, false, false>(Mh, 2, q + a * N3, q + a * N3, vol, t);
  wave_sync();
  if (tau == 0.0) return;   // uniform over the cell's lanes
  // div at the Gauss points: sum_b hinv_b (D along b, S along the others) p_b
  if (act) {
    sweep1<N, false, false>(D, 0, p, T, 1.0, t);
    cfence();
    sweep1<N, false, false>(S, 0, p + N3, T + N3, 1.0, t);
    cfence();
    sweep1<N, false, false>(S, 0, p + 2 * N3, T + 2 * N3, 1.0, t);
  }
  wave_sync();
  if (act) {
    sweep1<N, false, false>(S, 1, T, T, 1.0, t);
    cfence();
    sweep1<N, false, false>(D, 1, T + N3, T + N3, 1.0, t);
    cfence();
    sweep1<N, false, false>(S, 1, T + 2 * N3, T + 2 * N3, 1.0, t);
  }
  wave_sync();
  // along z on this lane's line: the divergence at the points, times tau vol w_i w_j w_k,
  // then the transposed z sweeps: T_1 = S^T dq, T_2 = D^T dq
  if (act) {
    const int a = t % N, b = t / N;
    const int base = b * N + a;
    constexpr int N2 = N * N;
    double v0[N], v1[N], v2[N], dq[N];
#pragma unroll
    for (int m = 0; m < N; ++m) {
      v0[m] = T[base + m * N2];
      v1[m] = T[N3 + base + m * N2];
      v2[m] = T[2 * N3 + base + m * N2];
    }
    const double sw = tau * vol * w[a] * w[b];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double r0 = 0, r2 = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        r0 = fma(S[i * N + m], fma(hinv[0], v0[m], hinv[1] * v1[m]), r0);
        r2 = fma(D[i * N + m], v2[m], r2);
      }
      dq[i] = sw * w[i] * fma(hinv[2], r2, r0);
    }
    cfence();
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double rs = 0, rd = 0;
#pragma unroll
      for (int m = 0; m < N; ++m) {
        rs = fma(S[m * N + i], dq[m], rs);
        rd = fma(D[m * N + i], dq[m], rd);
      }
      T[N3 + base + i * N2] = rs;
      T[2 * N3 + base + i * N2] = rd;
    }
  }
  wave_sync();
  if (act) {
    sweep1<N, true, false>(S, 1, T + N3, T, 1.0, t);              // S^T_y S^T_z dq (component 0)
    cfence();
    sweep1<N, true, false>(D, 1, T + N3, T + N3, 1.0, t);         // D^T_y S^T_z dq (component 1, in place)
    cfence();
    sweep1<N, true, false>(S, 1, T + 2 * N3, T + 2 * N3, 1.0, t); // S^T_y D^T_z dq (component 2, in place)
  }
  wave_sync();
  if (act) {
    sweep1<N, true, true>(D, 0, T, q, hinv[0], t);
    cfence();
    sweep1<N, true, true>(S, 0, T + N3, q + N3, hinv[1], t);
    cfence();
    sweep1<N, true, true>(S, 0, T + 2 * N3, q + 2 * N3, hinv[2], t);
  }
  wave_sync();
}

// z = M_e^{-1} r = (1/vol) Mi_z Mi_y Mi_x r per component (the y and z sweeps in place)
template <int N>
__device__ __forceinline__ void proj_precond(const double* tg, const double* tb, const double* r, double* z,
                                             double vol, int t, bool act) {
  constexpr int N3 = N * N * N;
  const auto Mi = tab_ptr<N, 6>(tg + V3Tab{N}.Mi(), tb + V3Tab{N}.Mi());
  if (act)
#pragma unroll 1
    for (int a = 0; a < 3; ++a) sweep1<N, false, false>(Mi, 0, r + a * N3, z + a * N3, 1.0, t);
  wave_sync();
  if (act)
#pragma unroll 1
    for (int a = 0; a < 3; ++a) sweep1<N, false, false>(Mi, 1, z + a * N3, z + a * N3, 1.0, t);
  wave_sync();
  if (act)
#pragma unroll 1
    for (int a = 0; a < 3; ++a) sweep1<N, false, false>(Mi, 2, z + a * N3, z + a * N3, 1.0 / vol, t);
  wave_sync();
}

template <int N, int WAVES>
__global__ void __launch_bounds__(64 * WAVES) k_v3_projection(
    const double* __restrict__ rhs, double* __restrict__ xg, const CartGeom<double> g,
    const double* __restrict__ tab, const double* __restrict__ taus, double rtol, int max_iter, int* iters,
    int64_t ncells) {
  using P = PPack<N>;
  constexpr int N2 = P::N2, N3 = P::N3, V = P::V, SS = P::SS, CPW = P::CPW;
  __shared__ double s_tab[V3Shape<N>::TABN];
  __shared__ double s_all[WAVES * CPW * P::SLICE];
  for (int e = threadIdx.x; e < V3Shape<N>::TABN; e += blockDim.x) s_tab[e] = tab[e];
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  const int slot = lane / SS, t = lane % SS;
  const int64_t cell = (static_cast<int64_t>(blockIdx.x) * WAVES + wave) * CPW + slot;
  // a cell's lanes leave together; the group sums read only lanes of the same cell
  if (cell >= ncells) return;
  const bool act = t < N2;
  double* r = s_all + (wave * CPW + slot) * P::SLICE;
  double* p = r + V;    // x for the first apply
  double* q = p + V;
  double* T = q + V;    // temporary of the apply; z between the preconditioner and the p update
  const int64_t Nd = ncells * N3;
  const CellIdx ci = cell_of(g, cell);
  const double vol = ci.h[0] * ci.h[1] * ci.h[2];
  const double hinv[3] = {1.0 / ci.h[0], 1.0 / ci.h[1], 1.0 / ci.h[2]};
  const double tau = taus[cell];
  double xr[3 * N];    // x of this lane's nodes t + N^2 j, in registers
  double bb = 0;
#pragma unroll
  for (int j = 0; j < 3 * N; ++j) xr[j] = 0.0;
  if (act)
#pragma unroll
    for (int j = 0; j < 3 * N; ++j) {
      const int e = t + N2 * j;
      const int64_t at = (e / N3) * Nd + cell * N3 + e % N3;
      xr[j] = xg[at];
      p[e] = xr[j];
      const double b = rhs[at];
      r[e] = b;
      bb = fma(b, b, bb);
    }
  bb = group_sum<SS>(bb);
  wave_sync();
  proj_apply<N>(tab, s_tab, p, q, T, hinv, vol, tau, t, act);
  double rr = 0;
  if (act)
#pragma unroll
    for (int j = 0; j < 3 * N; ++j) {
      const int e = t + N2 * j;
      const double d = r[e] - q[e];
      r[e] = d;
      rr = fma(d, d, rr);
    }
  rr = group_sum<SS>(rr);
  wave_sync();
  const double tol2 = rtol * rtol * bb;
  int it = 0;
  if (rr > tol2) {
    proj_precond<N>(tab, s_tab, r, T, vol, t, act);
    double rz = 0;
    if (act)
#pragma unroll
      for (int j = 0; j < 3 * N; ++j) {
        const int e = t + N2 * j;
        p[e] = T[e];
        rz = fma(r[e], T[e], rz);
      }
    rz = group_sum<SS>(rz);
    wave_sync();
    while (it < max_iter) {
      proj_apply<N>(tab, s_tab, p, q, T, hinv, vol, tau, t, act);
      double pq = 0;
      if (act)
#pragma unroll
        for (int j = 0; j < 3 * N; ++j) pq = fma(p[t + N2 * j], q[t + N2 * j], pq);
      pq = group_sum<SS>(pq);
      if (!(pq > 0)) break;    // breakdown (only for a non-positive tau)
      const double alpha = rz / pq;
      rr = 0;
      if (act)
#pragma unroll
        for (int j = 0; j < 3 * N; ++j) {
          const int e = t + N2 * j;
          xr[j] = fma(alpha, p[e], xr[j]);
          const double d = fma(-alpha, q[e], r[e]);
          r[e] = d;
          rr = fma(d, d, rr);
        }
      rr = group_sum<SS>(rr);
      ++it;
      wave_sync();
      if (rr <= tol2) break;
      proj_precond<N>(tab, s_tab, r, T, vol, t, act);
      double rz1 = 0;
      if (act)
#pragma unroll
        for (int j = 0; j < 3 * N; ++j) rz1 = fma(r[t + N2 * j], T[t + N2 * j], rz1);
      rz1 = group_sum<SS>(rz1);
      const double beta = rz1 / rz;
      rz = rz1;
      if (act)
#pragma unroll
        for (int j = 0; j < 3 * N; ++j) {
          const int e = t + N2 * j;
          p[e] = fma(beta, p[e], T[e]);
        }
      wave_sync();
    }
  }
  if (act)
#pragma unroll
    for (int j = 0; j < 3 * N; ++j) {
      const int e = t + N2 * j;
      xg[(e / N3) * Nd + cell * N3 + e % N3] = xr[j];
    }
  if (iters && t == 0) iters[cell] = it;
}

template <int N>
dgmf_status div_n(bool grad, const CartGeom<double>& g, const double* tab, const double* in, double* out,
                  int64_t ncells, hipStream_t s) {
  constexpr int CPW = DivPack<N>::CPW;
  const int64_t waves = (ncells + CPW - 1) / CPW;
  if (grad) {
    constexpr int W = GradPack<N>::WAVES;
    const int64_t blocks = (waves + W - 1) / W;
    if (blocks > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "v3: too many cells for one launch");
    hipLaunchKernelGGL((k_v3_gradient<N, W>), dim3(static_cast<unsigned>(blocks)), dim3(64 * W), 0, s, in, out, g,
                       tab, ncells);
    DGMF_LAUNCH_CHECK("k_v3_gradient");
  } else {
    constexpr int W = DivPack<N>::WAVES;
    const int64_t blocks = (waves + W - 1) / W;
    if (blocks > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "v3: too many cells for one launch");
    hipLaunchKernelGGL((k_v3_divergence<N, W>), dim3(static_cast<unsigned>(blocks)), dim3(64 * W), 0, s, in, out, g,
                       tab, ncells);
    DGMF_LAUNCH_CHECK("k_v3_divergence");
  }
  return DGMF_OK;
}

dgmf_status div_dispatch(int n, bool grad, const CartGeom<double>& g, const double* tab, const double* in,
                         double* out, int64_t ncells, hipStream_t s) {
  switch (n) {
    case 2: return div_n<2>(grad, g, tab, in, out, ncells, s);
    case 3: return div_n<3>(grad, g, tab, in, out, ncells, s);
    case 4: return div_n<4>(grad, g, tab, in, out, ncells, s);
    case 5: return div_n<5>(grad, g, tab, in, out, ncells, s);
    case 6: return div_n<6>(grad, g, tab, in, out, ncells, s);
    case 7: return div_n<7>(grad, g, tab, in, out, ncells, s);
    case 8: return div_n<8>(grad, g, tab, in, out, ncells, s);
    default: return fail(DGMF_UNSUPPORTED, "v3: n = %d not built", n);
  }
}

template <int N>
dgmf_status tau_n(const CartGeom<double>& g, const double* tab, const double* u, double zeta, double dt, double* tau,
                  int64_t ncells, hipStream_t s) {
  const int64_t blocks = (ncells + 3) / 4;
  hipLaunchKernelGGL((k_v3_tau<N>), dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, u, g, tab, zeta, dt, tau,
                     ncells);
  DGMF_LAUNCH_CHECK("k_v3_tau");
  return DGMF_OK;
}

template <int N>
dgmf_status proj_n(const CartGeom<double>& g, const double* tab, const double* tau, const double* rhs, double* x,
                   double rtol, int max_iter, int* iters, int64_t ncells, hipStream_t s) {
  constexpr int W = PPack<N>::WAVES, CPW = PPack<N>::CPW;
  const int64_t waves = (ncells + CPW - 1) / CPW;
  const int64_t blocks = (waves + W - 1) / W;
  if (blocks > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "v3: too many cells for one launch");
  hipLaunchKernelGGL((k_v3_projection<N, W>), dim3(static_cast<unsigned>(blocks)), dim3(64 * W), 0, s, rhs, x, g,
                     tab, tau, rtol, max_iter, iters, ncells);
  DGMF_LAUNCH_CHECK("k_v3_projection");
  return DGMF_OK;
}

}  // namespace

dgmf_status launch_v3_divergence(int n, const CartGeom<double>& g, const double* tab, const double* u, double* out,
                                 int64_t ncells, hipStream_t s) {
  return div_dispatch(n, false, g, tab, u, out, ncells, s);
}

dgmf_status launch_v3_gradient(int n, const CartGeom<double>& g, const double* tab, const double* p, double* out,
                               int64_t ncells, hipStream_t s) {
  return div_dispatch(n, true, g, tab, p, out, ncells, s);
}

dgmf_status launch_v3_tau(int n, const CartGeom<double>& g, const double* tab, const double* u, double zeta,
                          double dt, double* tau, int64_t ncells, hipStream_t s) {
  if ((ncells + 3) / 4 > 0x7fffffff) return fail(DGMF_UNSUPPORTED, "v3: too many cells for one launch");
  switch (n) {
    case 2: return tau_n<2>(g, tab, u, zeta, dt, tau, ncells, s);
    case 3: return tau_n<3>(g, tab, u, zeta, dt, tau, ncells, s);
    case 4: return tau_n<4>(g, tab, u, zeta, dt, tau, ncells, s);
    case 5: return tau_n<5>(g, tab, u, zeta, dt, tau, ncells, s);
    case 6: return tau_n<6>(g, tab, u, zeta, dt, tau, ncells, s);
    case 7: return tau_n<7>(g, tab, u, zeta, dt, tau, ncells, s);
    case 8: return tau_n<8>(g, tab, u, zeta, dt, tau, ncells, s);
    default: return fail(DGMF_UNSUPPORTED, "v3: n = %d not built", n);
  }
}

bool v3_projection_supported(int n) { return n >= 2 && n <= 7; }

dgmf_status launch_v3_projection(int n, const CartGeom<double>& g, const double* tab, const double* tau,
                                 const double* rhs, double* x, double rtol, int max_iter, int* iters, int64_t ncells,
                                 hipStream_t s) {
  switch (n) {
    case 2: return proj_n<2>(g, tab, tau, rhs, x, rtol, max_iter, iters, ncells, s);
    case 3: return proj_n<3>(g, tab, tau, rhs, x, rtol, max_iter, iters, ncells, s);
    case 4: return proj_n<4>(g, tab, tau, rhs, x, rtol, max_iter, iters, ncells, s);
    case 5: return proj_n<5>(g, tab, tau, rhs, x, rtol, max_iter, iters, ncells, s);
    case 6: return proj_n<6>(g, tab, tau, rhs, x, rtol, max_iter, iters, ncells, s);
    case 7: return proj_n<7>(g, tab, tau, rhs, x, rtol, max_iter, iters, ncells, s);
    default: return fail(DGMF_UNSUPPORTED, "projection: degree %d not built (k <= 6)", n - 1);
  }
}

}  // namespace dgmf
