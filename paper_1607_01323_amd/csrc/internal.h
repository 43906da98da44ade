// Internal declarations of libdgmf (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <string>
#include <vector>

#include "dgmf.h"

namespace dgmf {

constexpr int kMinDegree = 1;
constexpr int kMaxDegree = 7;
constexpr int kMaxConvPoints = 12;

// Geometry of a mesh whose metric is stored at every quadrature point.
template <typename T>
struct MetricGeom {
  int nx, ny, nz;
  int per[3];
  int neu;         // bit 2d+s: the boundary side (d, s) is homogeneous Neumann (no face term)
  const T* cm;     // [ncells][7][n^3]: G00 G01 G02 G11 G12 G22 (w detJ J^-1 J^-T), w detJ
  const T* fm;     // [ncells][3][7][n^2]: high face of each direction: wdA, vL(3), vR(3)
  const T* ftau;   // [ncells][3]: penalty geometry of those faces
  const T* lm;     // low boundary faces of non-periodic directions, [faces][7][n^2]
  const T* ltau;
  int lbase[3];    // first low-boundary face of direction d
  T mu, nu, pen;   // mass, diffusion, penalty scale s
  const T* tab;    // S, D, Dg (n x n), l'(0), l'(1), w, E0, E1 (n)
};

struct ConvGeom {
  int nx, ny, nz;
  int per[3];
  int neu;             // bit 2d+s: the boundary side (d, s) is an outflow (Neumann) side
  const double* h[3];
  const double* hinv[3];
  const double* tab;   // S[nq*n], D[nq*n], w[nq], Mh^{-1}[n*n] (k+1-point 1D mass, inverted), GLL nodes[n]
  int S, D, w, Mi;     // offsets into tab
  // curved cells (both null on affine meshes): per quadrature point
  //   cmet[cell][3e+b][q]   = w_q adj(J)_eb  (q = (qz nq + qy) nq + qx)
  //   fmet[cell][3f+r][pq]  = w_q1 w_q2 (adj J)_{d r} on face f = 2d+s, normal along +xi_d
  //                          (pq = q2 nq + q1; t1 = y for d = 0 else x, t2 = y for d = 2 else z)
  const double* cmet;
  const double* fmet;
};

// ---------------------------------------------------------------- errors ---
dgmf_status fail(dgmf_status st, const char* fmt, ...);
void clear_error();

#define DGMF_HIP_TRY(expr)                                                          \
  do {                                                                              \
    hipError_t e_ = (expr);                                                         \
    if (e_ != hipSuccess)                                                           \
      return ::dgmf::fail(e_ == hipErrorOutOfMemory ? DGMF_OOM : DGMF_HIP_ERROR,    \
                          "%s failed: %s", #expr, hipGetErrorString(e_));           \
  } while (0)

#define DGMF_LAUNCH_CHECK(name)                                                     \
  do {                                                                              \
    hipError_t e_ = hipGetLastError();                                              \
    if (e_ != hipSuccess)                                                           \
      return ::dgmf::fail(DGMF_HIP_ERROR, "launch of %s failed: %s", name,          \
                          hipGetErrorString(e_));                                   \
  } while (0)

// ----------------------------------------------------------- 1D tables ---
// Nodal basis on the Gauss-Lobatto nodes of degree k over [0,1] evaluated on
// an nq-point Gauss rule.  Everything is computed here from the Legendre
// three-term recurrence by Newton's method in long double.
struct Tables1D {
  int k = 0, n = 0, nq = 0;
  std::vector<double> nodes;   // n GLL nodes on [0,1]
  std::vector<double> gll_w;   // n integrals of the Lagrange polynomials
  std::vector<double> xq, wq;  // nq Gauss points / weights on [0,1], sum w = 1
  std::vector<double> S, D;    // nq x n: l_j(x_q), l_j'(x_q) (row q)
  std::vector<double> Mhat;    // n x n: sum_q w_q l_i l_j  (1D reference mass)
  std::vector<double> Khat;    // n x n: sum_q w_q l_i' l_j' (1D reference stiffness)
  std::vector<double> g0, g1;  // n: l_j'(0), l_j'(1)
};
void gauss_legendre01(int nq, std::vector<double>& x, std::vector<double>& w);
void gll_nodes01(int k, std::vector<double>& x);
void lagrange_eval(const std::vector<double>& nodes, double x, double* val, double* der);
void make_tables(int k, int nq, Tables1D& t);

// ------------------------------------------------------ device buffers ---
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  dgmf_status alloc(size_t nbytes);
  dgmf_status upload(const void* host, size_t nbytes);
  void release();
  ~DevBuf() { release(); }
};

// ------------------------------------------------------------- kernels ---
// Geometry of an axis-aligned box mesh seen by the Cartesian kernels.  The
// per-direction arrays are indexed by the cell coordinate along that axis.
template <typename T>
struct CartGeom {
  int nx, ny, nz;
  int per[3];
  int neu;            // bit 2d+s: the boundary side (d, s) is homogeneous Neumann (no face term)
  const T* h[3];      // cell size
  const T* hinv[3];   // 1 / cell size
  const T* tp[3];     // w_d / h_d: contribution of direction d to tau_e / (s (k+1)^2)
  const T* x0[3];     // low vertex coordinate
  T pen;              // s (k+1)^2
  T mu, nu;           // mass and diffusion coefficients
  const T* tab;       // Mhat[n*n], Khat[n*n], g0[n], g1[n], S[nq*n], wq[nq], xq[nq], nodes[n], Xhat[n*n]
  int xcomb;          // 1: uniform x spacing, Xhat = Khat + (mu hx^2/nu) Mhat (or Mhat if nu = 0) is valid
  int allper;         // 1: every direction periodic
  const T* utab;      // uniform periodic meshes: pre-scaled line operators (UTab), else null
};

// Pre-scaled tables of a uniform, fully periodic mesh: there every face has
// the same geometry, so the own-cell part of each face flux folds into one
// n x n line matrix per direction.  Per direction d: A_d (n*n), G1_d, G0_d,
// g0s_d, g1s_d (n each), c_d; then E1, E0 (n each) and Mhat (n*n).
struct UTab {
  int n;
  __host__ __device__ int dir(int d) const { return d * (n * n + 4 * n + 1); }
  __host__ __device__ int A(int d) const { return dir(d); }
  __host__ __device__ int G1(int d) const { return dir(d) + n * n; }
  __host__ __device__ int G0(int d) const { return dir(d) + n * n + n; }
  __host__ __device__ int g0s(int d) const { return dir(d) + n * n + 2 * n; }
  __host__ __device__ int g1s(int d) const { return dir(d) + n * n + 3 * n; }
  __host__ __device__ int c(int d) const { return dir(d) + n * n + 4 * n; }
  __host__ __device__ int E1() const { return dir(3); }
  __host__ __device__ int E0() const { return dir(3) + n; }
  __host__ __device__ int Mh() const { return dir(3) + 2 * n; }
  __host__ __device__ int size() const { return dir(3) + 2 * n + n * n; }
};

// Offsets into the device table of an SIPG operator.
struct TabLayout {
  int n, nq;
  __host__ __device__ int mhat() const { return 0; }
  __host__ __device__ int khat() const { return n * n; }
  __host__ __device__ int g0() const { return 2 * n * n; }
  __host__ __device__ int g1() const { return 2 * n * n + n; }
  __host__ __device__ int S() const { return 2 * n * n + 2 * n; }
  __host__ __device__ int wq() const { return S() + nq * n; }
  __host__ __device__ int xq() const { return wq() + nq; }
  __host__ __device__ int nodes() const { return xq() + nq; }
  __host__ __device__ int xhat() const { return nodes() + n; }
  // Mhat^{-1} Khat and the Mhat^{-1} images of l'(0), l'(1), e_0, e_{n-1}
  __host__ __device__ int ktil() const { return xhat() + n * n; }
  __host__ __device__ int g0t() const { return ktil() + n * n; }
  __host__ __device__ int g1t() const { return g0t() + n; }
  __host__ __device__ int e0t() const { return g1t() + n; }
  __host__ __device__ int e1t() const { return e0t() + n; }
  __host__ __device__ int size() const { return e1t() + n; }
};

// Constant lattice map x = m p of a sheared box (on = 0: identity).
struct Shear {
  double m[9];
  double det;
  int on;
};

dgmf_status launch_node_coords(int n, const CartGeom<double>& g, const Shear& sh, double* xyz, int64_t ncells,
                               hipStream_t s);
dgmf_status launch_qp_coords(int n, int nq, const CartGeom<double>& g, const Shear& sh, double* xyz,
                             int64_t ncells, hipStream_t s);
dgmf_status launch_integrate(int n, int nq, const CartGeom<double>& g, const Shear& sh, const double* f, double* b,
                             int64_t ncells, hipStream_t s);
// Curved cells: node (quadrature = false) or Gauss-point (true) positions of
// the deformed box (amplitude amp, origin lo, lengths len); the load vector
// with the point weights w_q det J_q of the stored cell metric cm (n_q = k+1,
// S the n_q x n interpolation table).
dgmf_status launch_curved_coords(int n, int nq, bool quadrature, const CartGeom<double>& g, const double lo[3],
                                 const double len[3], double amp, double* xyz, int64_t ncells, hipStream_t s);
dgmf_status launch_integrate_curved(int n, const double* S, const double* cm, const double* f, double* b,
                                    int64_t ncells, hipStream_t s);

// Chebyshev-Jacobi step fused into the store of an operator apply: with x_k
// the apply's input and y = H x_k, the kernel overwrites dst (holding x_{k-1})
// with x_{k+1} = x_k + c1 (x_k - x_{k-1}) + c2 dinv (b - y); prev_zero reads
// x_{k-1} as zero (Saad, Iterative Methods for Sparse Linear Systems,
// Alg. 12.1 written as a three-term recurrence on x).
template <typename T>
struct ChebEpi {
  const T* b;
  const T* dinv;
  T c1, c2;
  int prev_zero;
};
template <typename T>
dgmf_status launch_sipg_cart_cheb(int n, const CartGeom<T>& g, const T* xk, T* dst, const ChebEpi<T>& epi,
                                  const int* stop, hipStream_t s);

// Operator apply; when partials is not null, also writes per-block partial
// sums of <src, dst>, sum(dst) and sum(src) to partials[4*block + 0..2].
// stop: optional device flag; when non-zero the launch does nothing (used by
// CG to idle the remaining kernels of a batch once it has finished).
template <typename T>
dgmf_status launch_sipg_cart_apply(int n, const CartGeom<T>& g, const T* src, T* dst, int64_t ncells,
                                   double* partials, const int* stop, hipStream_t s);
template <typename T>
dgmf_status launch_sipg_cart_diag(int n, const CartGeom<T>& g, T* diag, int64_t ncells, hipStream_t s);
// Grid size of the apply kernel (also the number of partial-sum rows it writes).
int sipg_cart_blocks(int n, const CartGeom<double>& g);
// Queries (once per device) the occupancy of every axis-aligned apply variant
// of degree n - 1, which the launch plans use.
void sipg_cart_prime(int n);

// Apply with the metric stored at the quadrature points; partials/stop as
// above, metric_apply_blocks(n, nx, ny, nz) partial rows.
int metric_apply_blocks(int n, int nx, int ny, int nz);
template <typename T>
dgmf_status launch_sipg_metric_apply(int n, const MetricGeom<T>& g, const T* src, T* dst, double* partials,
                                     const int* stop, hipStream_t s);
// The apply with the Chebyshev step of ChebEpi fused into its store (dst holds
// x_{k-1} on entry, xk is x_k).
template <typename T>
dgmf_status launch_sipg_metric_cheb(int n, const MetricGeom<T>& g, const T* xk, T* dst, const ChebEpi<T>& epi,
                                    const int* stop, hipStream_t s);
template <typename TO>
dgmf_status launch_sipg_metric_diag(int n, const MetricGeom<double>& g, TO* diag, hipStream_t s);
// Fills cm, fm, ftau, lm, ltau of a lattice mesh with J = Sh diag(h_c).
dgmf_status launch_metric_fill(int n, const MetricGeom<double>& g, const double* const x0[3], const double* const h[3],
                               const double shinv[9], double shdet, const double* wq, double* cm, double* fm,
                               double* ftau, double* lm, double* ltau, hipStream_t s);

// Fills the same arrays for iso-parametric curved cells (the interpolated box
// deformation of amplitude amp); ctab: GLL nodes, S, D, l(0), l(1), l'(0),
// l'(1), Gauss weights; taue: scratch of one double per cell.
dgmf_status launch_metric_fill_curved(int n, const MetricGeom<double>& g, const double* const x0[3],
                                      const double* const h[3], const double lo[3], const double len[3], double amp,
                                      const double* ctab, double* taue, double* cm, double* fm, double* ftau,
                                      double* lm, double* ltau, hipStream_t s);

dgmf_status launch_to_f32(const double* a, float* b, int64_t n, hipStream_t s);
// Layout of the metric tables: S, D, Dg = D S^{-1} (n x n), l'(0), l'(1), Gauss
// weights w, and the Lagrange basis on the Gauss points at 0 and at 1 (n each).
constexpr int metric_tab_size(int n) { return 3 * n * n + 5 * n; }

bool conv_supported(int n, int nq);
// C = C(U); with step, C = U - dt M^{-1} C(U) instead (explicit convective substep).
dgmf_status launch_conv_fwd(int n, int nq, const ConvGeom& g, const double* U, double* C, int64_t ncells,
                            bool step, double dt, hipStream_t s);
dgmf_status launch_conv_vjp(int n, int nq, const ConvGeom& g, const double* U, const double* W, double* G,
                            int64_t ncells, hipStream_t s);
// V3c divergence (grad = false: [3][N] -> [N]) or gradient (grad = true:
// [N] -> [3][N]) on curved cells, with a ConvGeom of n_q = n points and its metric
dgmf_status launch_curv_v3(int n, bool grad, const ConvGeom& g, const double* in, double* out, int64_t ncells,
                           hipStream_t s);
// div-div penalty (proj = false: tau from u, zeta, dt) or local projection
// (proj = true: x from taus, rhs, x, rtol, max_iter, iters) on curved cells, with
// the ConvGeom of n_q = n points (tab + Mi: S^{-1}) and wdet the SIPG cell metric
dgmf_status launch_curv_cell(int n, bool proj, const ConvGeom& g, const double* wdet, const double* u, double zeta,
                             double dt, double* tau, const double* taus, const double* rhs, double* x, double rtol,
                             int max_iter, int* iters, int64_t ncells, hipStream_t s);
// curved-cell metric of the convective operator (ConvGeom::cmet, fmet); off:
// offsets into tab of the GLL nodes, S, D, the Gauss weights, l(0) l(1), l'(0) l'(1)
dgmf_status launch_conv_fill_curved(int n, int nq, const double* const x0[3], const double* const h[3],
                                    const double lo[3], const double len[3], double amp, int nx, int ny,
                                    int64_t ncells, const double* tab, const int off[6], double* cmet, double* fmet,
                                    hipStream_t s);

// dst = M^{-1} src or dst = M src on nfields consecutive scalar fields of a
// curved mesh, with the per-point weights m_q = w_q det J_q of the stored cell
// metric cm; tab = [S | S^T | S^{-T} | S^{-1}].  src and dst may be the same array.
template <typename T>
dgmf_status launch_point_mass(int n, const T* tab, const T* cm, const T* src, T* dst, int64_t ncells, int nfields,
                              bool inverse, hipStream_t s);
// dst = M^{-1} src (inverse: table the n x n inverse 1D mass, jscale =
// 1/|det shear|) or dst = M src (table the 1D mass, jscale = |det shear|) on
// nfields consecutive scalar fields of an affine mesh (k+1 Gauss points).
// src and dst may be the same array.
template <typename T>
dgmf_status launch_block_mass(int n, const CartGeom<T>& g, T jscale, const T* table, const T* src, T* dst,
                              int64_t ncells, int nfields, bool inverse, hipStream_t s);

// Variant V3c operators on axis-aligned box meshes (fp64).  Table layout
// (V3Tab): Mh, Ch (Ch[i][j] = int l_i' l_j), Mh^{-1}, S, D (Gauss rule of
// k+1 points, row q), all n x n, then the Gauss weights w (n) and the
// integrals of the Lagrange basis gw (n).
struct V3Tab {
  int n;
  __host__ __device__ int Mh() const { return 0; }
  __host__ __device__ int Ch() const { return n * n; }
  __host__ __device__ int Mi() const { return 2 * n * n; }
  __host__ __device__ int S() const { return 3 * n * n; }
  __host__ __device__ int D() const { return 4 * n * n; }
  __host__ __device__ int w() const { return 5 * n * n; }
  __host__ __device__ int gw() const { return 5 * n * n + n; }
  // viscous coupling: Kh (int l_i' l_j'), Dn (l_j'(x_i) at the nodes), l'(0), l'(1)
  __host__ __device__ int Kh() const { return 5 * n * n + 2 * n; }
  __host__ __device__ int Dn() const { return 6 * n * n + 2 * n; }
  __host__ __device__ int g0() const { return 7 * n * n + 2 * n; }
  __host__ __device__ int g1() const { return 7 * n * n + 3 * n; }
  __host__ __device__ int size() const { return 7 * n * n + 4 * n; }
};
dgmf_status launch_v3_divergence(int n, const CartGeom<double>& g, const double* tab, const double* u, double* out,
                                 int64_t ncells, hipStream_t s);
dgmf_status launch_v3_gradient(int n, const CartGeom<double>& g, const double* tab, const double* p, double* out,
                               int64_t ncells, hipStream_t s);
dgmf_status launch_v3_tau(int n, const CartGeom<double>& g, const double* tab, const double* u, double zeta,
                          double dt, double* tau, int64_t ncells, hipStream_t s);
// out += nu C(u), the component coupling of the symmetric-gradient viscous
// operator (u, out: [3][N]); see eps.hip.
dgmf_status launch_eps_coupling(int n, const CartGeom<double>& g, const double* tab, const double* u, double* out,
                                double nu, int64_t ncells, hipStream_t s);
// out += nu C(u) on iso-parametric curved cells (the coupling of the same
// operator, Jacobians in closed form from the box deformation; see conv.hip).
// g: tables S, D, w at the k+1 Gauss points; off_*: offsets into g.tab of
// the GLL nodes, l(0) l(1) and l'(0) l'(1).
dgmf_status launch_eps_curved(int n, const ConvGeom& g, const double* const x0[3], const double* const h[3],
                              const double lo[3], const double len[3], double amp, int off_nodes, int off_e,
                              int off_gd, const double* u, double* out, double nu, int64_t ncells, hipStream_t s);
// H_eps u of an SIPG operator on affine or curved cells (u, out: [3][N]); device already current
dgmf_status viscous_apply_any(dgmf_op op, const double* u, double* out, hipStream_t stream);
bool v3_projection_supported(int n);
dgmf_status launch_v3_projection(int n, const CartGeom<double>& g, const double* tab, const double* tau,
                                 const double* rhs, double* x, double rtol, int max_iter, int* iters, int64_t ncells,
                                 hipStream_t s);
// Inverse of the 1D reference mass S^T W S (square S: n_q = k+1) as
// S^{-1} W^{-1} S^{-T}, row-major n x n; false when S is singular.
bool inverse_mass_1d(const Tables1D& t, std::vector<double>& out);

// Geometric multigrid transfers between a fine box mesh and the mesh with
// every even cell count halved: coarse counts, fine counts in x and y, and
// the ratio (1 or 2) per direction.  The transfer table holds, per direction
// d and child s, the n x n matrix E_d[s][i][a] = l_a((s + xi_i) / 2) (the
// identity in E_d[0] when direction d is not halved): [d][s][i][a].
struct MgXfer {
  int cnx, cny, cnz;
  int fnx, fny;
  int r[3];
};
template <typename T>
dgmf_status launch_mg_prolong(int n, const MgXfer& x, const T* xc, T* xf, const T* etab, const int* stop,
                              hipStream_t s);   // xf += P xc
template <typename T>
dgmf_status launch_mg_restrict(int n, const MgXfer& x, const T* bf, const T* tf, T* bc, const T* etab,
                               const int* stop, hipStream_t s);   // bc = P^T (bf - tf)
template <typename T>
dgmf_status launch_mg_cast_in(const double* r, T* b, int64_t N, const int* stop, hipStream_t s);
template <typename T>
dgmf_status launch_mg_cast_out(const T* x, double* z, int64_t N, hipStream_t s);
template <typename T>
dgmf_status launch_mg_diag(const double* diag, T* dinv, T* dsq, int64_t N, hipStream_t s);
// x = scale dinv b
template <typename T>
dgmf_status launch_mg_jacobi(const T* b, const T* dinv, T* x, double scale, int64_t N, const int* stop,
                             hipStream_t s);
// dst = xk + c1 (xk - dst) + c2 dinv (b - t)  (dst read as zero when prev_zero)
template <typename T>
dgmf_status launch_mg_cheb_vec(const T* xk, T* dst, const T* b, const T* t, const T* dinv, double c1, double c2,
                               bool prev_zero, int64_t N, const int* stop, hipStream_t s);
// Cached multigrid hierarchy of an SIPG operator (built by the CG code).
struct MgHierarchy;
void mg_destroy(MgHierarchy* h);

// Dispatch over the two SIPG apply kernels (tables of axis-aligned cells or
// metric stored at the quadrature points), and the number of partial rows the
// apply writes.
template <typename T>
dgmf_status sipg_apply(dgmf_op op, const T* src, T* dst, double* partials, const int* stop, hipStream_t s);
dgmf_status sipg_diag64(dgmf_op op, double* diag, hipStream_t s);
// The fused apply + Chebyshev step on axis-aligned operators; DGMF_UNSUPPORTED
// for operators with the stored metric (callers then apply and update apart).
template <typename T>
dgmf_status sipg_cheb(dgmf_op op, const T* xk, T* dst, const ChebEpi<T>& epi, const int* stop, hipStream_t s);
int64_t sipg_apply_blocks(dgmf_op op);

}  // namespace dgmf

// --------------------------------------------------------------- handles ---
struct dgmf_mesh_ {
  dgmf_box_desc desc{};
  int device = 0;
  int64_t ncells = 0, ndofs = 0;
  std::vector<double> verts[3];
  dgmf::DevBuf geo64, geo32;       // x0, h, 1/h, tp per direction (fp64 / fp32)
  dgmf::CartGeom<double> g64{};    // geometry pointers (coefficients unset)
  dgmf::CartGeom<float> g32{};
  dgmf::Tables1D tab;              // tables with n_q = k+1
  dgmf::DevBuf tab64;
  dgmf::Shear shear{{1, 0, 0, 0, 1, 0, 0, 0, 1}, 1.0, 0};
  // stored quadrature-point geometry (store_qp_metric): fp64 and fp32 copies
  dgmf::DevBuf met64, met32, mtab64, mtab32;
  dgmf::MetricGeom<double> mg64{};   // coefficients unset
  dgmf::MetricGeom<float> mg32{};
  dgmf::DevBuf minv64, minv32;     // inverse 1D mass (n x n) for dgmf_inverse_mass_apply
  dgmf::DevBuf mh32;               // 1D mass in fp32 (the fp64 one heads v3tab)
  dgmf::DevBuf v3tab;              // V3Tab tables (fp64)
  dgmf::DevBuf pmt64, pmt32;       // curved cells: S, S^T, S^{-T}, S^{-1} for the point-weight mass
  // curved cells: tables and per-point metric (n_q = k+1) of the V3c divergence and
  // gradient, filled on their first call
  dgmf::DevBuf qtab, qmet;
  dgmf::ConvGeom qgeo{};
  // curved cells: 1D tables of the viscous coupling (no per-point data), set up on first use;
  // eoff: offsets of the GLL nodes, l(0) l(1) and l'(0) l'(1) in etab
  dgmf::DevBuf etab;
  dgmf::ConvGeom egeo{};
  int eoff[3] = {0, 0, 0};
  int nops = 0;                    // live operators built on this mesh
};

struct dgmf_op_ {
  int kind = 0;                    // 1 = SIPG, 2 = convective
  dgmf_mesh mesh = nullptr;
  dgmf_sipg_desc sipg{};
  int nq = 0;
  dgmf::Tables1D tab;
  dgmf::DevBuf tab64, tab32;
  dgmf::DevBuf utab64, utab32;     // uniform periodic meshes only
  dgmf::CartGeom<double> g64{};
  dgmf::CartGeom<float> g32{};
  dgmf::DevBuf ctab;               // convective tables
  dgmf::DevBuf cmet;               // convective metric of curved cells (cell part, then face part)
  dgmf::ConvGeom cgeo{};
  dgmf::MetricGeom<double> mg64{};   // metric path (mesh->desc.store_qp_metric)
  dgmf::MetricGeom<float> mg32{};
  bool metric = false;
  dgmf::DevBuf diag64;             // SIPG operators: diag(H) in fp64, computed at create
  dgmf::MgHierarchy* mgh = nullptr;   // multigrid levels, built on first use
  // largest Ritz value of the Chebyshev preconditioner's Lanczos run, kept for
  // later solves with the same precision, step count, seed and projection
  struct {
    int valid = 0, dtype = 0, steps = 0, project = 0;
    uint64_t seed = 0;
    double theta = 0.0;
  } lz;
};
