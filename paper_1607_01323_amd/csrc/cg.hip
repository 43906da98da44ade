// Preconditioned conjugate gradients on the SIPG operator (Sec. 5.1).
//
// All scalars of the iteration live on the device: per-block partial sums are
// written by the vector kernels (and by the operator apply's epilogue), a
// single-workgroup kernel reduces them in a fixed order (deterministic) and
// advances the recurrence, and every later kernel of the iteration reads the
// new scalar from device memory.  A status word ends the iteration on the
// device: once it is non-zero every remaining kernel of the batch returns at
// once, so the host only reads the state every `check_every` iterations while
// the iteration count stays exact.
//
// Preconditioners: point Jacobi (fp64), or the Chebyshev acceleration of
// point Jacobi (Saad, Iterative Methods for Sparse Linear Systems, Alg. 12.1)
// from a zero start in fp32 or fp64, whose interval [lambda/range, lambda]
// comes from Lanczos on D^{-1/2} H D^{-1/2} (Sec. 5.1: Chebyshev smoothing
// with the matrix diagonal, eigenvalue estimates from a Krylov start-up).
// Singular problems (periodic Laplacian) are solved on zero-mean vectors by
// projecting b and every operator product (Sec. 5.1).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>
#include <type_traits>
#include <vector>

#include "internal.h"

namespace dgmf {
namespace {

constexpr int RUNNING = 0, CONVERGED = 1;
constexpr int kVecBlocks = 2048;   // grid of the vector kernels (grid-stride loops)
constexpr int kMaxLanczos = 64;

struct CgState {
  double rz;        // <r, z>
  double alpha, beta;
  double mean_q;    // mean of H p when projecting
  double rr;        // ||r||^2
  double tol2;      // (rtol ||b||)^2
  double bnorm2;    // ||b||^2 (projected)
  double mean_b;    // mean of b when projecting
  double lz_alpha[kMaxLanczos];
  double lz_beta[kMaxLanczos];
  double lz_tmp;
  int iter, status, max_iter, project, flexible;
};

enum Mode { M_BSUM, M_BNORM, M_QMEAN, M_INIT, M_ALPHA, M_BETA, M_LZ_MEAN, M_LZ_NORM, M_LZ_ALPHA, M_LZ_BETA };

// ------------------------------------------------------- reductions -----
template <int K>
__device__ __forceinline__ void block_partials(double (&v)[K], double* __restrict__ partials, int blk) {
  __shared__ double red[K][4];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_down(v[k], o, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) red[k][w] = v[k];
  __syncthreads();
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < K; ++k) partials[4 * blk + k] = red[k][0] + red[k][1] + red[k][2] + red[k][3];
  __syncthreads();
}

// One workgroup of 1024 threads: sums nparts partial rows in a fixed order,
// then thread 0 advances the scalar recurrence of `mode`.
__global__ void __launch_bounds__(1024) k_scalar(CgState* st, const double* __restrict__ partials, int nparts,
                                                 int mode, int64_t N, int step, int stopmask) {
  if (stopmask && st->status != RUNNING) return;
  __shared__ double sh[4][1024];
  double a[4] = {0, 0, 0, 0};
  for (int b = threadIdx.x; b < nparts; b += 1024)
#pragma unroll
    for (int k = 0; k < 4; ++k) a[k] += partials[4 * b + k];
#pragma unroll
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = a[k];
  __syncthreads();
  for (int s = 512; s > 0; s >>= 1) {
    if (threadIdx.x < s)
#pragma unroll
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x != 0) return;
  const double s0 = sh[0][0], s1 = sh[1][0], s2 = sh[2][0];
  const double invN = 1.0 / static_cast<double>(N);
  switch (mode) {
    case M_BSUM:   // s0 = sum b, s1 = sum x0^2 (finiteness only)
      st->mean_b = st->project ? s0 * invN : 0.0;
      if (!isfinite(s0) || !isfinite(s1)) st->status = DGMF_NONFINITE;
      break;
    case M_BNORM:  // s0 = ||b_projected||^2
      st->bnorm2 = s0;
      break;
    case M_QMEAN:  // s1 = sum(H x0)
      st->mean_q = st->project ? s1 * invN : 0.0;
      break;
    case M_INIT:   // s0 = <r,z>, s1 = <r,r>
      st->rz = s0;
      st->rr = s1;
      st->iter = 0;
      if (!isfinite(s1) || !isfinite(st->bnorm2)) st->status = DGMF_NONFINITE;
      else if (s1 <= st->tol2) st->status = CONVERGED;
      else if (st->max_iter <= 0) st->status = DGMF_NOT_CONVERGED;   // no iteration allowed: x stays x0
      else if (!(s0 > 0)) st->status = isfinite(s0) ? DGMF_BREAKDOWN : DGMF_NONFINITE;
      break;
    case M_ALPHA: {  // s0 = <p,Hp>, s1 = sum(Hp), s2 = sum(p)
      const double mq = st->project ? s1 * invN : 0.0;
      const double pq = s0 - (st->project ? s1 * s2 * invN : 0.0);
      st->mean_q = mq;
      if (!(pq > 0)) {
        st->status = isfinite(pq) ? DGMF_BREAKDOWN : DGMF_NONFINITE;
        break;
      }
      st->alpha = st->rz / pq;
      break;
    }
    case M_BETA: {  // s0 = <r,z> (new), s1 = <r,r>, s2 = <z, q - mean_q>
      st->iter += 1;
      st->rr = s1;
      if (!isfinite(s1)) { st->status = DGMF_NONFINITE; break; }
      if (s1 <= st->tol2) { st->status = CONVERGED; break; }
      if (st->iter >= st->max_iter) { st->status = DGMF_NOT_CONVERGED; break; }
      if (!(s0 > 0)) { st->status = isfinite(s0) ? DGMF_BREAKDOWN : DGMF_NONFINITE; break; }
      // Polak-Ribiere: <z+, r+ - r> = -alpha <z+, q~> since r+ = r - alpha q~
      st->beta = st->flexible ? -st->alpha * s2 / st->rz : s0 / st->rz;
      st->rz = s0;
      break;
    }
    case M_LZ_MEAN:  // s0 = sum v
      st->lz_tmp = st->project ? s0 * invN : 0.0;
      break;
    case M_LZ_NORM:  // s0 = ||v||^2
      st->lz_tmp = 1.0 / sqrt(s0);
      break;
    case M_LZ_ALPHA:
      st->lz_alpha[step] = s0;
      break;
    case M_LZ_BETA:
      st->lz_beta[step] = sqrt(s0);
      break;
  }
}

#define GRID_STRIDE(i, N) \
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < (N); i += static_cast<int64_t>(gridDim.x) * blockDim.x)

// sum b, sum x0^2
__global__ void __launch_bounds__(256) k_bsum(const double* __restrict__ b, const double* __restrict__ x, int64_t N,
                                              double* partials) {
  double v[2] = {0, 0};
  GRID_STRIDE(i, N) {
    v[0] += b[i];
    v[1] += x[i] * x[i];
  }
  block_partials<2>(v, partials, blockIdx.x);
}

// bp = b - mean_b; ||bp||^2
__global__ void __launch_bounds__(256) k_bproj(const double* __restrict__ b, double* __restrict__ bp, int64_t N,
                                               const CgState* st, double* partials) {
  const double m = st->mean_b;
  double v[1] = {0};
  GRID_STRIDE(i, N) {
    const double t = b[i] - m;
    bp[i] = t;
    v[0] += t * t;
  }
  block_partials<1>(v, partials, blockIdx.x);
}

// tol2 = rtol^2 ||bp||^2 (host passes rtol^2)
__global__ void k_set_tol(CgState* st, double rtol2, int max_iter) {
  st->tol2 = rtol2 * st->bnorm2;
  st->max_iter = max_iter;
}

// r = bp - (q - mean_q); optionally z = dinv r and partials <r,z>, <r,r>
__global__ void __launch_bounds__(256) k_init_r(const double* __restrict__ bp, const double* __restrict__ q,
                                                double* __restrict__ r, const double* __restrict__ dinv,
                                                double* __restrict__ z, int64_t N, const CgState* st,
                                                double* partials) {
  if (st->status != RUNNING) return;
  const double mq = st->mean_q;
  double v[2] = {0, 0};
  GRID_STRIDE(i, N) {
    const double ri = bp[i] - (q[i] - mq);
    r[i] = ri;
    v[1] += ri * ri;
    if (z) {
      const double zi = dinv[i] * ri;
      z[i] = zi;
      v[0] += ri * zi;
    }
  }
  block_partials<2>(v, partials, blockIdx.x);
}

// x += alpha p; r -= alpha (q - mean_q); Jacobi: z = dinv r and partials
// <r,z>, <r,r>, <z, q - mean_q> (the last for the flexible beta)
__global__ void __launch_bounds__(256) k_update(double* __restrict__ x, double* __restrict__ r,
                                                const double* __restrict__ p, const double* __restrict__ q,
                                                const double* __restrict__ dinv, double* __restrict__ z, int64_t N,
                                                const CgState* st, double* partials) {
  if (st->status != RUNNING) return;
  const double a = st->alpha, mq = st->mean_q;
  double v[3] = {0, 0, 0};
  GRID_STRIDE(i, N) {
    x[i] = fma(a, p[i], x[i]);
    const double qi = q[i] - mq;
    const double ri = fma(-a, qi, r[i]);
    r[i] = ri;
    v[1] += ri * ri;
    if (z) {
      const double zi = dinv[i] * ri;
      z[i] = zi;
      v[0] += ri * zi;
      v[2] += zi * qi;
    }
  }
  if (z) block_partials<3>(v, partials, blockIdx.x);
}

// k_update on element pairs (16-byte loads and stores; every vector 16-byte
// aligned), the odd last element by the first thread of the grid
__global__ void __launch_bounds__(256) k_update2(double* __restrict__ x, double* __restrict__ r,
                                                 const double* __restrict__ p, const double* __restrict__ q,
                                                 const double* __restrict__ dinv, double* __restrict__ z, int64_t N,
                                                 const CgState* st, double* partials) {
  if (st->status != RUNNING) return;
  const double a = st->alpha, mq = st->mean_q;
  double v[3] = {0, 0, 0};
  auto one = [&](double& xi, double& ri, double& zi, double pi, double qi, double di) {
    xi = fma(a, pi, xi);
    const double qm = qi - mq;
    ri = fma(-a, qm, ri);
    v[1] += ri * ri;
    if (z) {
      zi = di * ri;
      v[0] += ri * zi;
      v[2] += zi * qm;
    }
  };
  const int64_t N2 = N >> 1;
  double2* x2 = reinterpret_cast<double2*>(x);
  double2* r2 = reinterpret_cast<double2*>(r);
  double2* z2 = reinterpret_cast<double2*>(z);
  const double2* p2 = reinterpret_cast<const double2*>(p);
  const double2* q2 = reinterpret_cast<const double2*>(q);
  const double2* d2 = reinterpret_cast<const double2*>(dinv);
  GRID_STRIDE(i, N2) {
    double2 xv = x2[i], rv = r2[i];
    const double2 pv = p2[i], qv = q2[i];
    double2 dv = make_double2(0.0, 0.0), zv;
    if (z) dv = d2[i];
    one(xv.x, rv.x, zv.x, pv.x, qv.x, dv.x);
    one(xv.y, rv.y, zv.y, pv.y, qv.y, dv.y);
    x2[i] = xv;
    r2[i] = rv;
    if (z) z2[i] = zv;
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) {
    const int64_t k = N - 1;
    double zk = 0.0;
    one(x[k], r[k], zk, p[k], q[k], z ? dinv[k] : 0.0);
    if (z) z[k] = zk;
  }
  if (z) block_partials<3>(v, partials, blockIdx.x);
}

// p = z + beta p on element pairs, as k_update2
__global__ void __launch_bounds__(256) k_update_p2(double* __restrict__ p, const double* __restrict__ z, int64_t N,
                                                   const CgState* st, int first) {
  if (st->status != RUNNING) return;
  const double b = first ? 0.0 : st->beta;
  const int64_t N2 = N >> 1;
  double2* p2 = reinterpret_cast<double2*>(p);
  const double2* z2 = reinterpret_cast<const double2*>(z);
  GRID_STRIDE(i, N2) {
    const double2 zv = z2[i];
    double2 pv = first ? make_double2(0.0, 0.0) : p2[i];
    pv.x = fma(b, pv.x, zv.x);
    pv.y = fma(b, pv.y, zv.y);
    p2[i] = pv;
  }
  if ((N & 1) && blockIdx.x == 0 && threadIdx.x == 0) p[N - 1] = first ? z[N - 1] : fma(b, p[N - 1], z[N - 1]);
}

// p = z + beta p  (first = 1: p = z)
__global__ void __launch_bounds__(256) k_update_p(double* __restrict__ p, const double* __restrict__ z, int64_t N,
                                                  const CgState* st, int first) {
  if (st->status != RUNNING) return;
  const double b = first ? 0.0 : st->beta;
  GRID_STRIDE(i, N) p[i] = first ? z[i] : fma(b, p[i], z[i]);
}

__global__ void __launch_bounds__(256) k_recip(const double* __restrict__ d, double* __restrict__ dinv, int64_t N) {
  GRID_STRIDE(i, N) dinv[i] = 1.0 / d[i];
}

// ------------------------------------------------ Chebyshev (T = f32/f64) -
template <typename T>
__global__ void __launch_bounds__(256) k_cast_recip(const double* __restrict__ d, T* __restrict__ dinv,
                                                    T* __restrict__ dsq, int64_t N) {
  GRID_STRIDE(i, N) {
    const double v = 1.0 / d[i];
    dinv[i] = static_cast<T>(v);
    if (dsq) dsq[i] = static_cast<T>(sqrt(v));
  }
}

// When the preconditioner's last kernel writes z64 it also writes the partials
// <r,z>, <r,r>, <z, q - mean_q> (q = null at the initial residual).
__device__ __forceinline__ void final_terms(double (&v)[3], double ri, double zi, const double* __restrict__ q,
                                            int64_t i, double mq) {
  v[0] += ri * zi;
  v[1] += ri * ri;
  if (q) v[2] += zi * (q[i] - mq);
}

// z already holds M^{-1} r: the partials of the preconditioned update
__global__ void __launch_bounds__(256) k_mass_out(const double* __restrict__ r, const double* __restrict__ z,
                                                  const double* __restrict__ q, int64_t N, const CgState* st,
                                                  double* partials) {
  if (st->status != RUNNING) return;
  const double mq = st->mean_q;
  double v[3] = {0, 0, 0};
  GRID_STRIDE(i, N) final_terms(v, r[i], z[i], q, i, mq);
  block_partials<3>(v, partials, blockIdx.x);
}

// res = T(r); d = dinv res / theta; zc = d   (degree 1: z64 = d directly)
template <typename T>
__global__ void __launch_bounds__(256) k_cheb_init(const double* __restrict__ r, T* __restrict__ res,
                                                   T* __restrict__ d, T* __restrict__ zc, const T* __restrict__ dinv,
                                                   T inv_theta, double* __restrict__ z64, const double* __restrict__ q,
                                                   int64_t N, const CgState* st, double* partials) {
  if (st->status != RUNNING) return;
  const double mq = st->mean_q;
  double v[3] = {0, 0, 0};
  GRID_STRIDE(i, N) {
    const T ri = static_cast<T>(r[i]);
    const T di = dinv[i] * ri * inv_theta;
    if (z64) {
      const double zd = static_cast<double>(di);
      z64[i] = zd;
      final_terms(v, r[i], zd, q, i, mq);
    } else {
      res[i] = ri;
      d[i] = di;
      zc[i] = di;
    }
  }
  if (z64) block_partials<3>(v, partials, blockIdx.x);
}

// res -= t; d = c1 d + c2 dinv res; zc += d  (last step: z64 = zc)
template <typename T>
__global__ void __launch_bounds__(256) k_cheb_step(T* __restrict__ res, T* __restrict__ d, T* __restrict__ zc,
                                                   const T* __restrict__ t, const T* __restrict__ dinv, T c1, T c2,
                                                   const double* __restrict__ r, double* __restrict__ z64,
                                                   const double* __restrict__ q, int64_t N, const CgState* st,
                                                   double* partials) {
  if (st->status != RUNNING) return;
  const double mq = st->mean_q;
  double v[3] = {0, 0, 0};
  GRID_STRIDE(i, N) {
    const T ri = res[i] - t[i];
    const T di = fma(c1, d[i], c2 * dinv[i] * ri);
    const T zi = zc[i] + di;
    if (z64) {
      const double zd = static_cast<double>(zi);
      z64[i] = zd;
      final_terms(v, r[i], zd, q, i, mq);
    } else {
      res[i] = ri;
      d[i] = di;
      zc[i] = zi;
    }
  }
  if (z64) block_partials<3>(v, partials, blockIdx.x);
}

// z64 = x (the last Chebyshev iterate, fused path), with the partials of the
// preconditioned update
template <typename T>
__global__ void __launch_bounds__(256) k_cheb_fin(const T* __restrict__ x, const double* __restrict__ r,
                                                  double* __restrict__ z64, const double* __restrict__ q, int64_t N,
                                                  const CgState* st, double* partials) {
  if (st->status != RUNNING) return;
  const double mq = st->mean_q;
  double v[3] = {0, 0, 0};
  GRID_STRIDE(i, N) {
    const double zd = static_cast<double>(x[i]);
    z64[i] = zd;
    final_terms(v, r[i], zd, q, i, mq);
  }
  block_partials<3>(v, partials, blockIdx.x);
}

// ------------------------------------------------------------ Lanczos -----
// SplitMix64 (Steele, Lea & Flood 2014): output i = mix(seed + (i+1) gamma),
// mapped to [-1, 1) by its top 53 bits.
__global__ void __launch_bounds__(256) k_splitmix_uniform(double* __restrict__ v, uint64_t seed, int64_t N,
                                                          double* partials) {
  double s[1] = {0};
  GRID_STRIDE(i, N) {
    uint64_t z = seed + static_cast<uint64_t>(i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    const double u = 2.0 * static_cast<double>(z >> 11) * 0x1.0p-53 - 1.0;
    v[i] = u;
    s[0] += u;
  }
  block_partials<1>(s, partials, blockIdx.x);
}

// v64 -= mean; ||v64||^2
__global__ void __launch_bounds__(256) k_lz_center(double* __restrict__ v, int64_t N, const CgState* st,
                                                   double* partials) {
  const double m = st->lz_tmp;
  double s[1] = {0};
  GRID_STRIDE(i, N) {
    const double t = v[i] - m;
    v[i] = t;
    s[0] += t * t;
  }
  block_partials<1>(s, partials, blockIdx.x);
}

// v = T(v64 / ||v64||); vprev = 0
template <typename T>
__global__ void __launch_bounds__(256) k_lz_start(const double* __restrict__ v64, T* __restrict__ v,
                                                  T* __restrict__ vprev, int64_t N, const CgState* st) {
  const double s = st->lz_tmp;
  GRID_STRIDE(i, N) {
    v[i] = static_cast<T>(v64[i] * s);
    vprev[i] = T(0);
  }
}

// t = dsq v
template <typename T>
__global__ void __launch_bounds__(256) k_lz_scale(const T* __restrict__ v, const T* __restrict__ dsq,
                                                  T* __restrict__ t, int64_t N) {
  GRID_STRIDE(i, N) t[i] = dsq[i] * v[i];
}

// w = dsq w - beta_{j-1} vprev; partial <w, v>
template <typename T>
__global__ void __launch_bounds__(256) k_lz_w(T* __restrict__ w, const T* __restrict__ dsq, const T* __restrict__ v,
                                              const T* __restrict__ vprev, int64_t N, const CgState* st, int step,
                                              double* partials) {
  const T b = step > 0 ? static_cast<T>(st->lz_beta[step - 1]) : T(0);
  double s[1] = {0};
  GRID_STRIDE(i, N) {
    const T wi = fma(dsq[i], w[i], -b * vprev[i]);
    w[i] = wi;
    s[0] += static_cast<double>(wi) * static_cast<double>(v[i]);
  }
  block_partials<1>(s, partials, blockIdx.x);
}

// w -= alpha_j v; partial ||w||^2
template <typename T>
__global__ void __launch_bounds__(256) k_lz_orth(T* __restrict__ w, const T* __restrict__ v, int64_t N,
                                                 const CgState* st, int step, double* partials) {
  const T a = static_cast<T>(st->lz_alpha[step]);
  double s[1] = {0};
  GRID_STRIDE(i, N) {
    const T wi = fma(-a, v[i], w[i]);
    w[i] = wi;
    s[0] += static_cast<double>(wi) * static_cast<double>(wi);
  }
  block_partials<1>(s, partials, blockIdx.x);
}

// vprev = w / beta_j  (the caller then swaps the roles of v and vprev)
template <typename T>
__global__ void __launch_bounds__(256) k_lz_next(const T* __restrict__ w, T* __restrict__ vprev, int64_t N,
                                                 const CgState* st, int step) {
  const double b = st->lz_beta[step];
  const T s = static_cast<T>(b > 0 ? 1.0 / b : 0.0);
  GRID_STRIDE(i, N) vprev[i] = w[i] * s;
}

struct Layout {
  size_t state, partials, bp, r, z, p, q, dinv, v64;             // fp64 part
  size_t cdinv, cdsq, cres, cd, czc, ct;                       // precond dtype part
  size_t total;
};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

Layout make_layout(int64_t N, int64_t nparts, bool cheb, size_t es) {
  Layout L{};
  size_t off = 0;
  auto take = [&](size_t bytes) { size_t o = off; off = align256(off + bytes); return o; };
  L.state = take(sizeof(CgState));
  L.partials = take(sizeof(double) * 4 * nparts);
  const size_t v8 = sizeof(double) * N;
  L.bp = take(v8); L.r = take(v8); L.z = take(v8); L.p = take(v8); L.q = take(v8); L.dinv = take(v8);
  if (cheb) {
    L.v64 = take(v8);
    const size_t vc = es * N;
    L.cdinv = take(vc); L.cdsq = take(vc); L.cres = take(vc); L.cd = take(vc); L.czc = take(vc); L.ct = take(vc);
  }
  L.total = off;
  return L;
}

dgmf_status validate(dgmf_op op, const dgmf_cg_params* p) {
  if (!op || op->kind != 1) return fail(DGMF_INVALID, "cg: not an SIPG operator");
  if (!p) return fail(DGMF_INVALID, "cg: null params");
  if (!(p->rtol >= 0) || !std::isfinite(p->rtol)) return fail(DGMF_INVALID, "cg: rtol must be finite and >= 0");
  if (p->max_iter < 0) return fail(DGMF_INVALID, "cg: max_iter must be >= 0");
  if (p->precond < 0 || p->precond > 3) return fail(DGMF_INVALID, "cg: precond must be 0, 1, 2 or 3");
  if (p->precond == 1 || p->precond == 2) {
    if (p->precond_dtype != DGMF_F32 && p->precond_dtype != DGMF_F64)
      return fail(DGMF_INVALID, "cg: precond_dtype must be DGMF_F32 or DGMF_F64");
    if (p->cheb_degree < 1 || p->cheb_degree > 64) return fail(DGMF_INVALID, "cg: cheb_degree must be in 1..64");
    if (!(p->smoothing_range > 1)) return fail(DGMF_INVALID, "cg: smoothing_range must be > 1");
    if (p->lanczos_steps < 2 || p->lanczos_steps > kMaxLanczos)
      return fail(DGMF_INVALID, "cg: lanczos_steps must be in 2..%d", kMaxLanczos);
    if (!(p->lambda_safety >= 1)) return fail(DGMF_INVALID, "cg: lambda_safety must be >= 1");
  }
  if (p->precond == 2 && !(p->mg_coarse_tol >= 0 && p->mg_coarse_tol < 1))
    return fail(DGMF_INVALID, "cg: mg_coarse_tol must be in [0, 1)");
  if (p->precond == 2 && p->mg_graph != 0 && p->mg_graph != 1) return fail(DGMF_INVALID, "cg: mg_graph must be 0 or 1");
  return DGMF_OK;
}

int64_t nparts_for(dgmf_op op) {
  const int64_t a = sipg_apply_blocks(op);
  return a > kVecBlocks ? a : kVecBlocks;
}


dgmf_status launch_scalar(CgState* st, const double* partials, int nblk, int mode, int64_t N, int step, int stopmask,
                          hipStream_t s) {
  hipLaunchKernelGGL(k_scalar, dim3(1), dim3(1024), 0, s, st, partials, nblk, mode, N, step, stopmask);
  DGMF_LAUNCH_CHECK("k_scalar");
  return DGMF_OK;
}

// k-th smallest eigenvalue (k = 0..m-1) of the symmetric tridiagonal (a, b)
// by bisection on the Sturm sequence count, bracketed by Gershgorin discs.
double tridiag_eig(const double* a, const double* b, int m, int k) {
  double lo = 1e300, hi = -1e300;
  for (int i = 0; i < m; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i < m - 1 ? std::fabs(b[i]) : 0.0);
    lo = std::fmin(lo, a[i] - r);
    hi = std::fmax(hi, a[i] + r);
  }
  auto count_below = [&](double x) {
    int c = 0;
    double q = 1.0;
    for (int i = 0; i < m; ++i) {
      const double bb = i > 0 ? b[i - 1] * b[i - 1] : 0.0;
      q = a[i] - x - (i > 0 ? bb / q : 0.0);
      if (q == 0.0) q = -1e-300;
      if (q < 0) ++c;
    }
    return c;
  };
  for (int it = 0; it < 200 && hi - lo > 1e-15 * std::fmax(std::fabs(lo), std::fabs(hi)); ++it) {
    const double mid = 0.5 * (lo + hi);
    if (count_below(mid) >= k + 1) hi = mid; else lo = mid;
  }
  return hi;
}

// Chebyshev acceleration of Jacobi on [a, b] with an error polynomial of degree m
// (Saad, Alg. 12.1): d_0 = dinv r / theta; d_j = c1[j] d_{j-1} + c2[j] dinv r_j.
void cheb_coeffs(double a, double b, int m, double& inv_theta, std::vector<double>& c1, std::vector<double>& c2) {
  const double th = 0.5 * (a + b), de = 0.5 * (b - a), sigma = th / de;
  inv_theta = 1.0 / th;
  double rho = 1.0 / sigma;
  c1.assign(m, 0.0);
  c2.assign(m, 0.0);
  for (int j = 1; j < m; ++j) {
    const double rn = 1.0 / (2.0 * sigma - rho);
    c1[j] = rn * rho;
    c2[j] = 2.0 * rn / de;
    rho = rn;
  }
}

template <typename T>
struct LzBufs {
  T* dsq;
  T* v;
  T* vp;
  T* w;
  T* t;
  double* v64;
};

// Largest Ritz value of m Lanczos steps (no re-orthogonalisation) on
// D^{-1/2} H D^{-1/2} in precision T, start vector SplitMix64(seed) with its
// mean removed when st->project.
template <typename T>
dgmf_status lanczos_max(dgmf_op op, int64_t N, const LzBufs<T>& B, CgState* st, double* partials, int m,
                        uint64_t seed, hipStream_t s, double& theta) {
  T* v = B.v;
  T* vp = B.vp;
  const dim3 G(kVecBlocks), Bk(256);
  hipLaunchKernelGGL(k_splitmix_uniform, G, Bk, 0, s, B.v64, seed, N, partials);
  DGMF_LAUNCH_CHECK("k_splitmix_uniform");
  dgmf_status e = launch_scalar(st, partials, kVecBlocks, M_LZ_MEAN, N, 0, 0, s);
  if (e) return e;
  hipLaunchKernelGGL(k_lz_center, G, Bk, 0, s, B.v64, N, st, partials);
  DGMF_LAUNCH_CHECK("k_lz_center");
  if ((e = launch_scalar(st, partials, kVecBlocks, M_LZ_NORM, N, 0, 0, s))) return e;
  hipLaunchKernelGGL((k_lz_start<T>), G, Bk, 0, s, B.v64, v, vp, N, st);
  DGMF_LAUNCH_CHECK("k_lz_start");
  for (int j = 0; j < m; ++j) {
    hipLaunchKernelGGL((k_lz_scale<T>), G, Bk, 0, s, v, B.dsq, B.t, N);
    DGMF_LAUNCH_CHECK("k_lz_scale");
    if ((e = sipg_apply<T>(op, B.t, B.w, nullptr, nullptr, s))) return e;
    hipLaunchKernelGGL((k_lz_w<T>), G, Bk, 0, s, B.w, B.dsq, v, vp, N, st, j, partials);
    DGMF_LAUNCH_CHECK("k_lz_w");
    if ((e = launch_scalar(st, partials, kVecBlocks, M_LZ_ALPHA, N, j, 0, s))) return e;
    hipLaunchKernelGGL((k_lz_orth<T>), G, Bk, 0, s, B.w, v, N, st, j, partials);
    DGMF_LAUNCH_CHECK("k_lz_orth");
    if ((e = launch_scalar(st, partials, kVecBlocks, M_LZ_BETA, N, j, 0, s))) return e;
    hipLaunchKernelGGL((k_lz_next<T>), G, Bk, 0, s, B.w, vp, N, st, j);
    DGMF_LAUNCH_CHECK("k_lz_next");
    T* tmp = v; v = vp; vp = tmp;
  }
  double ha[kMaxLanczos], hb[kMaxLanczos];
  DGMF_HIP_TRY(hipMemcpyAsync(ha, st->lz_alpha, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  DGMF_HIP_TRY(hipMemcpyAsync(hb, st->lz_beta, sizeof(double) * m, hipMemcpyDeviceToHost, s));
  DGMF_HIP_TRY(hipStreamSynchronize(s));
  int mm = m;
  for (int j = 0; j < m; ++j) {
    if (!std::isfinite(ha[j])) { mm = j; break; }
    if (j < m - 1 && !(hb[j] > 0)) { mm = j + 1; break; }
  }
  if (mm < 1) return fail(DGMF_NONFINITE, "cg: eigenvalue estimate is not finite");
  theta = tridiag_eig(ha, hb, mm, mm - 1);
  if (!(theta > 0) || !std::isfinite(theta)) return fail(DGMF_BREAKDOWN, "cg: eigenvalue estimate %g <= 0", theta);
  return DGMF_OK;
}

// The i-th SplitMix64 output of a generator seeded with `seed`, as a double in [-1, 1).
double splitmix_uniform_host(uint64_t seed, int64_t i) {
  uint64_t z = seed + static_cast<uint64_t>(i + 1) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z = z ^ (z >> 31);
  return 2.0 * static_cast<double>(z >> 11) * 0x1.0p-53 - 1.0;
}

// z64 = x (precision T) and the partials <r,z>, <r,r>, <z, q - mean_q>.
template <typename T>
__global__ void __launch_bounds__(256) k_mg_out(const T* __restrict__ x, const double* __restrict__ r,
                                                double* __restrict__ z, const double* __restrict__ q, int64_t N,
                                                const CgState* st, double* partials) {
  if (st->status != RUNNING) return;
  const double mq = st->mean_q;
  double v[3] = {0, 0, 0};
  GRID_STRIDE(i, N) {
    const double zd = static_cast<double>(x[i]);
    z[i] = zd;
    final_terms(v, r[i], zd, q, i, mq);
  }
  block_partials<3>(v, partials, blockIdx.x);
}

}  // namespace

// ---------------------------------------------------------- multigrid ---
// One level of the hierarchy: its mesh and operator (the caller's on the
// finest level), seven vectors in the preconditioner precision (b, two
// alternating iterates, one spare used by the set-up, t = H x, dinv, dsq),
// the transfer to the next coarser level, and the Chebyshev parameters of its
// smoother (or of the coarse solver).
struct MgLevel {
  dgmf_mesh mesh = nullptr;
  dgmf_op op = nullptr;
  bool owned = false;
  int64_t N = 0;
  int nc[3] = {0, 0, 0};
  MgXfer xf{};
  DevBuf vec, etab;
  double lambda = 0, lo = 0, hi = 0, inv_theta = 0;
  int m = 0;
  int xout = 1;   // buffer (1 or 2) that holds the last V-cycle result
  std::vector<double> c1, c2;
  template <typename T>
  T* v(int k) { return static_cast<T*>(vec.p) + k * N; }
};

struct MgHierarchy {
  dgmf_cg_params key{};
  std::vector<MgLevel> lv;
  DevBuf scratch;
  // captured V-cycles (HIP graphs) keyed by the stop flag their kernels read,
  // and the private stream they are captured on
  hipStream_t cap = nullptr;
  std::vector<std::pair<const int*, hipGraphExec_t>> graphs;
  ~MgHierarchy() {
    for (auto& g : graphs) (void)hipGraphExecDestroy(g.second);
    if (cap) (void)hipStreamDestroy(cap);
    for (auto& l : lv)
      if (l.owned) {
        l.vec.release();
        l.etab.release();
        if (l.op) dgmf_op_destroy(l.op);
        if (l.mesh) dgmf_mesh_destroy(l.mesh);
      }
  }
};

void mg_destroy(MgHierarchy* h) { delete h; }

namespace {

bool mg_same(const dgmf_cg_params& a, const dgmf_cg_params& b) {
  return a.precond_dtype == b.precond_dtype && a.cheb_degree == b.cheb_degree &&
         a.smoothing_range == b.smoothing_range && a.lanczos_steps == b.lanczos_steps &&
         a.lambda_safety == b.lambda_safety && a.seed == b.seed && (a.project_mean != 0) == (b.project_mean != 0) &&
         a.mg_coarse_tol == b.mg_coarse_tol;
}

double coarse_tol(const dgmf_cg_params& p) { return p.mg_coarse_tol > 0 ? p.mg_coarse_tol : 1e-3; }

constexpr int kMaxCoarseDegree = 2000;

// Extreme Ritz values of fp64 Lanczos with full re-orthogonalisation on the
// coarsest level's D^{-1/2} H D^{-1/2} (host-driven; the level is small), the
// null vector D^{1/2} 1 deflated for singular problems.
dgmf_status coarse_interval(MgLevel& c, const std::vector<double>& diag, bool singular, uint64_t seed, double* dv,
                            double* dw, hipStream_t s, double& tmin, double& tmax) {
  const int64_t N = c.N;
  std::vector<double> sq(N), nul;
  for (int64_t i = 0; i < N; ++i) sq[i] = std::sqrt(diag[i]);
  if (singular) {
    double nn = 0;
    for (double v : sq) nn += v * v;
    nn = std::sqrt(nn);
    nul.resize(N);
    for (int64_t i = 0; i < N; ++i) nul[i] = sq[i] / nn;
  }
  auto dot = [&](const std::vector<double>& a, const std::vector<double>& b) {
    double r = 0;
    for (int64_t i = 0; i < N; ++i) r += a[i] * b[i];
    return r;
  };
  auto deflate = [&](std::vector<double>& w) {
    if (!singular) return;
    const double a = dot(nul, w);
    for (int64_t i = 0; i < N; ++i) w[i] -= a * nul[i];
  };
  auto normalise = [&](std::vector<double>& w) {
    const double nrm = std::sqrt(dot(w, w));
    for (auto& x : w) x /= nrm;
  };
  const int steps = static_cast<int>(std::min<int64_t>(64, N - (singular ? 1 : 0)));
  if (steps < 1) return fail(DGMF_UNSUPPORTED, "multigrid: coarse level too small");
  std::vector<std::vector<double>> V;
  std::vector<double> v(N), w(N), t(N), al, be;
  for (int64_t i = 0; i < N; ++i) v[i] = splitmix_uniform_host(seed, i);
  deflate(v);
  normalise(v);
  for (int j = 0; j < steps; ++j) {
    V.push_back(v);
    for (int64_t i = 0; i < N; ++i) t[i] = v[i] / sq[i];
    DGMF_HIP_TRY(hipMemcpyAsync(dv, t.data(), sizeof(double) * N, hipMemcpyHostToDevice, s));
    dgmf_status e = sipg_apply<double>(c.op, dv, dw, nullptr, nullptr, s);
    if (e) return e;
    DGMF_HIP_TRY(hipMemcpyAsync(w.data(), dw, sizeof(double) * N, hipMemcpyDeviceToHost, s));
    DGMF_HIP_TRY(hipStreamSynchronize(s));
    for (int64_t i = 0; i < N; ++i) w[i] /= sq[i];
    const double alpha = dot(w, v);
    deflate(w);
    for (int pass = 0; pass < 2; ++pass)
      for (const auto& u : V) {
        const double a = dot(u, w);
        for (int64_t i = 0; i < N; ++i) w[i] -= a * u[i];
      }
    al.push_back(alpha);
    const double beta = std::sqrt(dot(w, w));
    double scale = 0;
    for (double a : al) scale = std::fmax(scale, std::fabs(a));
    if (j == steps - 1 || beta <= 1e-8 * scale) break;
    be.push_back(beta);
    for (int64_t i = 0; i < N; ++i) v[i] = w[i] / beta;
    deflate(v);
    normalise(v);
  }
  const int m = static_cast<int>(al.size());
  be.resize(m);
  tmin = tridiag_eig(al.data(), be.data(), m, 0);
  tmax = tridiag_eig(al.data(), be.data(), m, m - 1);
  if (!(tmin > 0) || !(tmax >= tmin) || !std::isfinite(tmax))
    return fail(DGMF_BREAKDOWN, "multigrid: coarse eigenvalue estimates [%g, %g] are not positive", tmin, tmax);
  return DGMF_OK;
}

template <typename T>
dgmf_status mg_build(dgmf_op op, const dgmf_cg_params& prm, hipStream_t s, MgHierarchy*& out) {
  if (op->mesh->shear.on) return fail(DGMF_UNSUPPORTED, "multigrid: sheared meshes are not supported");
  auto* h = new (std::nothrow) MgHierarchy;
  if (!h) return fail(DGMF_OOM, "multigrid: host allocation failed");
  std::unique_ptr<MgHierarchy> guard(h);
  h->key = prm;
  const int n = op->mesh->tab.n;
  int c[3] = {op->mesh->desc.nx, op->mesh->desc.ny, op->mesh->desc.nz};
  {
    MgLevel f;
    f.mesh = op->mesh;
    f.op = op;
    f.N = op->mesh->ndofs;
    for (int d = 0; d < 3; ++d) f.nc[d] = c[d];
    h->lv.push_back(std::move(f));
  }
  for (;;) {
    int nxt[3];
    bool any = false;
    for (int d = 0; d < 3; ++d) {
      nxt[d] = c[d] % 2 == 0 ? c[d] / 2 : c[d];
      any = any || nxt[d] != c[d];
    }
    if (!any) break;
    dgmf_box_desc d = op->mesh->desc;
    d.nx = nxt[0];
    d.ny = nxt[1];
    d.nz = nxt[2];
    d.store_qp_metric = 0;
    d.curve_amp = 0.0;    // a curved finest level: the coarse levels are the undeformed box
    for (double& v : d.shear) v = 0.0;
    MgLevel l;
    l.owned = true;
    dgmf_status e = dgmf_mesh_create(&d, &l.mesh);
    if (e) return e;
    e = dgmf_sipg_create(l.mesh, &op->sipg, &l.op);
    if (e) {
      dgmf_mesh_destroy(l.mesh);
      return e;
    }
    l.N = l.mesh->ndofs;
    for (int k = 0; k < 3; ++k) l.nc[k] = nxt[k];
    h->lv.push_back(std::move(l));
    for (int k = 0; k < 3; ++k) c[k] = nxt[k];
  }
  const int L = static_cast<int>(h->lv.size());
  // transfer tables E_d[s][i][a] = l_a((s + xi_i) / r_d)
  const Tables1D& tb = op->mesh->tab;
  for (int l = 0; l + 1 < L; ++l) {
    MgLevel& f = h->lv[l];
    const MgLevel& g = h->lv[l + 1];
    f.xf = MgXfer{g.nc[0], g.nc[1], g.nc[2], f.nc[0], f.nc[1], {f.nc[0] / g.nc[0], f.nc[1] / g.nc[1], f.nc[2] / g.nc[2]}};
    std::vector<T> tab(6 * n * n, T(0));
    std::vector<double> val(n);
    for (int d = 0; d < 3; ++d)
      for (int sd = 0; sd < f.xf.r[d]; ++sd)
        for (int i = 0; i < n; ++i) {
          if (f.xf.r[d] == 1) {
            tab[(d * 2 + sd) * n * n + i * n + i] = T(1);
            continue;
          }
          lagrange_eval(tb.nodes, 0.5 * (sd + tb.nodes[i]), val.data(), nullptr);
          for (int a = 0; a < n; ++a) tab[(d * 2 + sd) * n * n + i * n + a] = static_cast<T>(val[a]);
        }
    dgmf_status e = f.etab.upload(tab.data(), tab.size() * sizeof(T));
    if (e) return e;
  }
  for (auto& l : h->lv) {
    dgmf_status e = l.vec.alloc(7 * l.N * sizeof(T));
    if (e) return e;
  }
  // scratch: CgState, partials, two fp64 vectors of the finest size
  const int64_t N0 = h->lv[0].N;
  const size_t o_part = align256(sizeof(CgState)), o_v64 = align256(o_part + sizeof(double) * 4 * kVecBlocks),
               o_d64 = align256(o_v64 + sizeof(double) * N0), total = align256(o_d64 + sizeof(double) * N0);
  dgmf_status e = h->scratch.alloc(total);
  if (e) return e;
  char* sc = static_cast<char*>(h->scratch.p);
  CgState* st = reinterpret_cast<CgState*>(sc);
  double* partials = reinterpret_cast<double*>(sc + o_part);
  double* v64 = reinterpret_cast<double*>(sc + o_v64);
  double* d64 = reinterpret_cast<double*>(sc + o_d64);
  CgState init{};
  init.project = prm.project_mean ? 1 : 0;
  DGMF_HIP_TRY(hipMemcpyAsync(st, &init, sizeof(init), hipMemcpyHostToDevice, s));
  for (int l = 0; l < L; ++l) {
    MgLevel& a = h->lv[l];
    const double* dg = static_cast<const double*>(a.op->diag64.p);   // computed at the level's create
    if ((e = launch_mg_diag<T>(dg, a.v<T>(5), a.v<T>(6), a.N, s))) return e;
    if (l + 1 < L) {
      LzBufs<T> B{a.v<T>(6), a.v<T>(0), a.v<T>(1), a.v<T>(2), a.v<T>(3), v64};
      double theta = 0;
      if ((e = lanczos_max<T>(a.op, a.N, B, st, partials, prm.lanczos_steps, prm.seed + l, s, theta))) return e;
      a.lambda = prm.lambda_safety * theta;
      a.lo = a.lambda / prm.smoothing_range;
      a.hi = a.lambda;
      a.m = prm.cheb_degree;
    } else {
      std::vector<double> dh(a.N);
      DGMF_HIP_TRY(hipMemcpyAsync(dh.data(), dg, sizeof(double) * a.N, hipMemcpyDeviceToHost, s));
      DGMF_HIP_TRY(hipStreamSynchronize(s));
      double tmin = 0, tmax = 0;
      if ((e = coarse_interval(a, dh, prm.project_mean != 0, prm.seed + l, v64, d64, s, tmin, tmax))) return e;
      a.lo = tmin / prm.lambda_safety;
      a.hi = prm.lambda_safety * tmax;
      a.lambda = a.hi;
      const double sigma = (a.hi + a.lo) / (a.hi - a.lo);
      const double m = std::ceil(std::acosh(1.0 / coarse_tol(prm)) / std::acosh(sigma));
      if (!(m <= kMaxCoarseDegree))
        return fail(DGMF_UNSUPPORTED, "multigrid: coarse Chebyshev would need %g steps (limit %d)", m,
                    kMaxCoarseDegree);
      a.m = std::max(1, static_cast<int>(m));
    }
    cheb_coeffs(a.lo, a.hi, a.m, a.inv_theta, a.c1, a.c2);
  }
  DGMF_HIP_TRY(hipStreamSynchronize(s));
  out = guard.release();
  return DGMF_OK;
}

dgmf_status mg_ensure(dgmf_op op, const dgmf_cg_params& prm, hipStream_t s) {
  if (op->mgh && mg_same(op->mgh->key, prm)) return DGMF_OK;
  if (op->mgh) {
    mg_destroy(op->mgh);
    op->mgh = nullptr;
  }
  MgHierarchy* h = nullptr;
  dgmf_status e = prm.precond_dtype == DGMF_F32 ? mg_build<float>(op, prm, s, h) : mg_build<double>(op, prm, s, h);
  if (e) return e;
  op->mgh = h;
  return DGMF_OK;
}

// One Chebyshev-Jacobi step on level a: buffer dst (holding x_{k-1}) becomes
// x_{k+1} from x_k in buffer src; fused into the apply where the operator
// allows it, else an apply into t and a vector update.
template <typename T>
dgmf_status cheb_step(MgLevel& a, int src, int dst, double c1, double c2, bool prev_zero, const int* stop,
                      hipStream_t s) {
  const T* b = a.v<T>(0);
  const T* dinv = a.v<T>(5);
  const ChebEpi<T> epi{b, dinv, static_cast<T>(c1), static_cast<T>(c2), prev_zero ? 1 : 0};
  dgmf_status e = sipg_cheb<T>(a.op, a.v<T>(src), a.v<T>(dst), epi, stop, s);
  if (e != DGMF_UNSUPPORTED) return e;
  clear_error();
  T* t = a.v<T>(4);
  if ((e = sipg_apply<T>(a.op, a.v<T>(src), t, nullptr, stop, s))) return e;
  return launch_mg_cheb_vec<T>(a.v<T>(src), a.v<T>(dst), b, t, dinv, c1, c2, prev_zero, a.N, stop, s);
}

// Chebyshev smoothing (or the coarse solve) on level a, from zero or from the
// iterate in buffer cur; on return cur names the buffer holding the result.
// Buffers 1 and 2 alternate as x_k and x_{k-1}.
template <typename T>
dgmf_status smooth(MgLevel& a, bool from_zero, int& cur, const int* stop, hipStream_t s) {
  dgmf_status e = DGMF_OK;
  int prev = 3 - cur;
  bool prev_zero = true;
  if (from_zero) {
    if ((e = launch_mg_jacobi<T>(a.v<T>(0), a.v<T>(5), a.v<T>(cur), a.inv_theta, a.N, stop, s))) return e;
  } else {
    // x_1 = x_0 + dinv (b - H x_0) / theta into the other buffer
    if ((e = cheb_step<T>(a, cur, prev, 0.0, a.inv_theta, true, stop, s))) return e;
    std::swap(cur, prev);
    prev_zero = false;
  }
  for (int j = 1; j < a.m; ++j) {
    if ((e = cheb_step<T>(a, cur, prev, a.c1[j], a.c2[j], prev_zero, stop, s))) return e;
    std::swap(cur, prev);
    prev_zero = false;
  }
  return DGMF_OK;
}

// x_l = V-cycle(b_l) on level l (Sec. 5.1): pre-smoothing from zero, residual
// restricted to the next level, its V-cycle prolongated and added,
// post-smoothing from the corrected x; the coarsest level runs the coarse
// Chebyshev from zero.  The result is left in buffer a.xout.
template <typename T>
dgmf_status vcycle(MgHierarchy& h, int l, const int* stop, hipStream_t s) {
  MgLevel& a = h.lv[l];
  const int L = static_cast<int>(h.lv.size());
  int cur = 1;
  dgmf_status e = smooth<T>(a, true, cur, stop, s);
  if (e) return e;
  if (l == L - 1) {
    a.xout = cur;
    return DGMF_OK;
  }
  MgLevel& c = h.lv[l + 1];
  const int n = a.mesh->tab.n;
  T* t = a.v<T>(4);
  if ((e = sipg_apply<T>(a.op, a.v<T>(cur), t, nullptr, stop, s))) return e;
  if ((e = launch_mg_restrict<T>(n, a.xf, a.v<T>(0), t, c.v<T>(0), static_cast<const T*>(a.etab.p), stop, s)))
    return e;
  if ((e = vcycle<T>(h, l + 1, stop, s))) return e;
  if ((e = launch_mg_prolong<T>(n, a.xf, c.v<T>(c.xout), a.v<T>(cur), static_cast<const T*>(a.etab.p), stop, s)))
    return e;
  if ((e = smooth<T>(a, false, cur, stop, s))) return e;
  a.xout = cur;
  return DGMF_OK;
}

constexpr size_t kMaxGraphs = 4;

// The whole V-cycle on stream s: launched kernel by kernel, or (graph) replayed
// from a HIP graph captured once per stop flag on the hierarchy's own stream.
// The coarse levels are launch-latency bound, and the graph removes the host
// launch gaps between their ~150 small kernels.  The V-cycle records no
// memset or copy, only kernels with fixed arguments.
template <typename T>
dgmf_status vcycle_run(MgHierarchy& h, const int* stop, bool graph, hipStream_t s) {
  if (!graph) return vcycle<T>(h, 0, stop, s);
  for (auto& g : h.graphs)
    if (g.first == stop) {
      DGMF_HIP_TRY(hipGraphLaunch(g.second, s));
      return DGMF_OK;
    }
  if (!h.cap) DGMF_HIP_TRY(hipStreamCreateWithFlags(&h.cap, hipStreamNonBlocking));
  DGMF_HIP_TRY(hipStreamBeginCapture(h.cap, hipStreamCaptureModeThreadLocal));
  dgmf_status e = vcycle<T>(h, 0, stop, h.cap);
  hipGraph_t gr = nullptr;
  const hipError_t ce = hipStreamEndCapture(h.cap, &gr);
  if (e) {
    if (gr) (void)hipGraphDestroy(gr);
    return e;
  }
  if (ce != hipSuccess || !gr)
    return fail(DGMF_HIP_ERROR, "multigrid: V-cycle capture failed: %s", hipGetErrorString(ce));
  hipGraphExec_t ex = nullptr;
  const hipError_t ie = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
  (void)hipGraphDestroy(gr);
  if (ie != hipSuccess) return fail(DGMF_HIP_ERROR, "multigrid: graph instantiation failed: %s", hipGetErrorString(ie));
  if (h.graphs.size() >= kMaxGraphs) {
    (void)hipGraphExecDestroy(h.graphs.front().second);
    h.graphs.erase(h.graphs.begin());
  }
  h.graphs.push_back({stop, ex});
  DGMF_HIP_TRY(hipGraphLaunch(ex, s));
  return DGMF_OK;
}

struct Solver {
  dgmf_op op;
  const dgmf_cg_params& prm;
  char* ws;
  Layout L;
  hipStream_t s;
  int64_t N, nparts;
  int n;
  CgState* st;
  double* partials;
  double cheb_inv_theta = 0;
  std::vector<double> c1, c2;
  double lambda = 0;

  template <typename V>
  V* at(size_t off) { return reinterpret_cast<V*>(ws + off); }

  dgmf_status scalar(int mode, int nblk, int step = 0, int stopmask = 1) {
    hipLaunchKernelGGL(k_scalar, dim3(1), dim3(1024), 0, s, st, partials, nblk, mode, N, step, stopmask);
    DGMF_LAUNCH_CHECK("k_scalar");
    return DGMF_OK;
  }

  template <typename T>
  dgmf_status apply(const T* src, T* dst, bool with_partials) {
    return sipg_apply<T>(op, src, dst, with_partials ? partials : nullptr, &st->status, s);
  }

  // Lanczos in precision T on D^{-1/2} H D^{-1/2}; fills lambda and the Chebyshev coefficients.
  template <typename T>
  dgmf_status lanczos_and_coeffs() {
    LzBufs<T> B{at<T>(L.cdsq), at<T>(L.cres), at<T>(L.cd), at<T>(L.czc), at<T>(L.ct), at<double>(L.v64)};
    double theta = 0;
    const int dt = std::is_same<T, float>::value ? DGMF_F32 : DGMF_F64;
    const int proj = prm.project_mean ? 1 : 0;
    auto& c = op->lz;
    if (c.valid && c.dtype == dt && c.steps == prm.lanczos_steps && c.seed == prm.seed && c.project == proj) {
      theta = c.theta;
    } else {
      dgmf_status e = lanczos_max<T>(op, N, B, st, partials, prm.lanczos_steps, prm.seed, s, theta);
      if (e) return e;
      c.valid = 1;
      c.dtype = dt;
      c.steps = prm.lanczos_steps;
      c.seed = prm.seed;
      c.project = proj;
      c.theta = theta;
    }
    lambda = prm.lambda_safety * theta;
    cheb_coeffs(lambda / prm.smoothing_range, lambda, prm.cheb_degree, cheb_inv_theta, c1, c2);
    return DGMF_OK;
  }

  // z64 = Chebyshev(r64) in precision T, with partials <r,z>, <r,r>, <z, q~>.
  template <typename T>
  dgmf_status cheb_apply(const double* r, double* z, const double* q) {
    const dim3 G(kVecBlocks), B(256);
    T* dinv = at<T>(L.cdinv);
    T* res = at<T>(L.cres);
    T* d = at<T>(L.cd);
    T* zc = at<T>(L.czc);
    T* t = at<T>(L.ct);
    const int m = prm.cheb_degree;
    hipLaunchKernelGGL((k_cheb_init<T>), G, B, 0, s, r, res, d, zc, dinv, static_cast<T>(cheb_inv_theta),
                       m == 1 ? z : nullptr, q, N, st, partials);
    DGMF_LAUNCH_CHECK("k_cheb_init");
    if (m > 1) {
      // the same polynomial in the three-term form
      // x_{j+1} = x_j + c1 (x_j - x_{j-1}) + c2 D^{-1} (r - H x_j), x_0 = 0,
      // x_1 = d, each step fused into the apply's store (5 vectors instead of
      // 10); the buffers of x_j and x_{j-1} swap after every step
      T* cur = d;
      T* prev = zc;
      for (int j = 1; j < m; ++j) {
        const ChebEpi<T> epi{res, dinv, static_cast<T>(c1[j]), static_cast<T>(c2[j]), j == 1 ? 1 : 0};
        dgmf_status e = sipg_cheb<T>(op, cur, prev, epi, &st->status, s);
        if (e) return e;
        T* tmp = cur;
        cur = prev;
        prev = tmp;
      }
      hipLaunchKernelGGL((k_cheb_fin<T>), G, B, 0, s, cur, r, z, q, N, st, partials);
      DGMF_LAUNCH_CHECK("k_cheb_fin");
      return DGMF_OK;
    }
    for (int j = 1; j < m; ++j) {
      dgmf_status e = apply<T>(d, t, false);
      if (e) return e;
      hipLaunchKernelGGL((k_cheb_step<T>), G, B, 0, s, res, d, zc, t, dinv, static_cast<T>(c1[j]),
                         static_cast<T>(c2[j]), r, j == m - 1 ? z : nullptr, q, N, st, partials);
      DGMF_LAUNCH_CHECK("k_cheb_step");
    }
    return DGMF_OK;
  }

  // z64 = V-cycle(r64) in precision T, with the same partials.
  template <typename T>
  dgmf_status mg_apply(const double* r, double* z, const double* q) {
    MgLevel& a = op->mgh->lv[0];
    dgmf_status e = launch_mg_cast_in<T>(r, a.v<T>(0), N, &st->status, s);
    if (e || (e = vcycle_run<T>(*op->mgh, &st->status, prm.mg_graph != 0, s))) return e;
    hipLaunchKernelGGL((k_mg_out<T>), dim3(kVecBlocks), dim3(256), 0, s, a.v<T>(a.xout), r, z, q, N, st, partials);
    DGMF_LAUNCH_CHECK("k_mg_out");
    return DGMF_OK;
  }

  // z = M^{-1} r (fp64; the preconditioner of the viscous step, Sec. 5.1), then the partials
  dgmf_status mass_apply(const double* r, double* z, const double* q) {
    const dgmf_mesh m = op->mesh;
    dgmf_status e;
    if (m->desc.curve_amp != 0.0)
      e = launch_point_mass<double>(n, static_cast<const double*>(m->pmt64.p), m->mg64.cm, r, z, m->ncells, 1, true,
                                    s);
    else
      e = launch_block_mass<double>(n, m->g64, 1.0 / std::fabs(m->shear.det), static_cast<const double*>(m->minv64.p),
                                    r, z, m->ncells, 1, true, s);
    if (e) return e;
    hipLaunchKernelGGL(k_mass_out, dim3(kVecBlocks), dim3(256), 0, s, r, z, q, N, st, partials);
    DGMF_LAUNCH_CHECK("k_mass_out");
    return DGMF_OK;
  }

  dgmf_status precond(const double* r, double* z, const double* q) {
    if (prm.precond == 3) return mass_apply(r, z, q);
    if (prm.precond == 2) {
      if (prm.precond_dtype == DGMF_F32) return mg_apply<float>(r, z, q);
      return mg_apply<double>(r, z, q);
    }
    if (prm.precond_dtype == DGMF_F32) return cheb_apply<float>(r, z, q);
    return cheb_apply<double>(r, z, q);
  }
};

// The solve proper, on a workspace laid out as L.  Every non-OK return is
// turned into out->status and a synchronised stream by the caller.
dgmf_status cg_run(dgmf_op op, const double* b, double* x, const dgmf_cg_params* params, char* ws,
                   const Layout& L, hipStream_t stream, dgmf_cg_result* out) {
  const int64_t N = op->mesh->ndofs;
  const bool cheb = params->precond == 1;
  const bool poly = params->precond != 0;   // preconditioner kernels write z and the partials
  dgmf_status e = DGMF_OK;
  Solver S{op, *params, ws, L, stream, N, nparts_for(op), op->mesh->desc.degree + 1,
           nullptr, nullptr};
  S.st = S.at<CgState>(L.state);
  S.partials = S.at<double>(L.partials);
  double* bp = S.at<double>(L.bp);
  double* r = S.at<double>(L.r);
  double* z = S.at<double>(L.z);
  double* p = S.at<double>(L.p);
  double* q = S.at<double>(L.q);
  double* dinv = S.at<double>(L.dinv);
  const double* diag = static_cast<const double*>(op->diag64.p);   // computed at create
  const dim3 G(kVecBlocks), B(256);
  const int napply = static_cast<int>(sipg_apply_blocks(op));
  auto t0 = std::chrono::steady_clock::now();

  // ---- set-up: state, diagonal, eigenvalue estimate
  CgState init{};
  init.project = params->project_mean ? 1 : 0;
  init.flexible = params->flexible ? 1 : 0;
  init.max_iter = params->max_iter;
  DGMF_HIP_TRY(hipMemcpyAsync(S.st, &init, sizeof(init), hipMemcpyHostToDevice, stream));
  hipLaunchKernelGGL(k_recip, G, B, 0, stream, diag, dinv, N);
  DGMF_LAUNCH_CHECK("k_recip");
  if (cheb) {
    if (params->precond_dtype == DGMF_F32) {
      hipLaunchKernelGGL((k_cast_recip<float>), G, B, 0, stream, diag, S.at<float>(L.cdinv), S.at<float>(L.cdsq), N);
      DGMF_LAUNCH_CHECK("k_cast_recip");
      e = S.lanczos_and_coeffs<float>();
    } else {
      hipLaunchKernelGGL((k_cast_recip<double>), G, B, 0, stream, diag, S.at<double>(L.cdinv), S.at<double>(L.cdsq),
                         N);
      DGMF_LAUNCH_CHECK("k_cast_recip");
      e = S.lanczos_and_coeffs<double>();
    }
    if (e) {
      (void)hipStreamSynchronize(stream);
      out->status = e;
      return e;
    }
    out->lambda_max = S.lambda;
  } else if (params->precond == 2) {
    if ((e = mg_ensure(op, *params, stream))) {
      out->status = e;
      return e;
    }
    out->lambda_max = op->mgh->lv[0].lambda;
  }
  // ---- initial residual
  hipLaunchKernelGGL(k_bsum, G, B, 0, stream, b, x, N, S.partials);
  DGMF_LAUNCH_CHECK("k_bsum");
  if ((e = S.scalar(M_BSUM, kVecBlocks, 0, 0))) return e;
  hipLaunchKernelGGL(k_bproj, G, B, 0, stream, b, bp, N, S.st, S.partials);
  DGMF_LAUNCH_CHECK("k_bproj");
  if ((e = S.scalar(M_BNORM, kVecBlocks, 0, 0))) return e;
  hipLaunchKernelGGL(k_set_tol, dim3(1), dim3(1), 0, stream, S.st, params->rtol * params->rtol, params->max_iter);
  DGMF_LAUNCH_CHECK("k_set_tol");
  if ((e = sipg_apply<double>(op, x, q, S.partials, nullptr, stream))) return e;
  if ((e = S.scalar(M_QMEAN, napply, 0, 0))) return e;
  if (poly) {
    hipLaunchKernelGGL(k_init_r, G, B, 0, stream, bp, q, r, dinv, static_cast<double*>(nullptr), N, S.st,
                       S.partials);
    DGMF_LAUNCH_CHECK("k_init_r");
    if ((e = S.precond(r, z, nullptr))) return e;
  } else {
    hipLaunchKernelGGL(k_init_r, G, B, 0, stream, bp, q, r, dinv, z, N, S.st, S.partials);
    DGMF_LAUNCH_CHECK("k_init_r");
  }
  if ((e = S.scalar(M_INIT, kVecBlocks))) return e;
  hipLaunchKernelGGL(k_update_p, G, B, 0, stream, p, z, N, S.st, 1);
  DGMF_LAUNCH_CHECK("k_update_p");
  CgState h{};
  DGMF_HIP_TRY(hipMemcpyAsync(&h, S.st, sizeof(h), hipMemcpyDeviceToHost, stream));
  DGMF_HIP_TRY(hipStreamSynchronize(stream));
  auto t1 = std::chrono::steady_clock::now();

  // ---- iteration
  const int batch = params->check_every > 0 ? params->check_every : 1;
  // pairs of elements per thread where x is 16-byte aligned (the workspace
  // vectors always are)
  const bool pairs = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
  while (h.status == RUNNING) {
    for (int k = 0; k < batch; ++k) {
      if ((e = S.apply<double>(p, q, true))) return e;
      if ((e = S.scalar(M_ALPHA, napply))) return e;
      if (pairs)
        hipLaunchKernelGGL(k_update2, G, B, 0, stream, x, r, p, q, dinv, poly ? static_cast<double*>(nullptr) : z, N,
                           S.st, S.partials);
      else
        hipLaunchKernelGGL(k_update, G, B, 0, stream, x, r, p, q, dinv, poly ? static_cast<double*>(nullptr) : z, N,
                           S.st, S.partials);
      DGMF_LAUNCH_CHECK("k_update");
      if (poly && (e = S.precond(r, z, q))) return e;
      if ((e = S.scalar(M_BETA, kVecBlocks))) return e;
      hipLaunchKernelGGL(k_update_p2, G, B, 0, stream, p, z, N, S.st, 0);
      DGMF_LAUNCH_CHECK("k_update_p");
    }
    DGMF_HIP_TRY(hipMemcpyAsync(&h, S.st, sizeof(h), hipMemcpyDeviceToHost, stream));
    DGMF_HIP_TRY(hipStreamSynchronize(stream));
  }
  auto t2 = std::chrono::steady_clock::now();
  out->iterations = h.iter;
  out->rel_residual = h.bnorm2 > 0 ? std::sqrt(h.rr / h.bnorm2) : 0.0;
  out->status = h.status == CONVERGED ? DGMF_OK : h.status;
  out->setup_s = std::chrono::duration<double>(t1 - t0).count();
  out->solve_s = std::chrono::duration<double>(t2 - t1).count();
  if (out->status != DGMF_OK) {
    static const char* names[] = {"OK", "INVALID", "HIP_ERROR", "OOM", "NOT_CONVERGED", "BREAKDOWN", "NONFINITE",
                                  "UNSUPPORTED"};
    return fail(static_cast<dgmf_status>(out->status), "cg_solve: %s after %d iterations (rel. residual %g)",
                names[out->status], out->iterations, out->rel_residual);
  }
  return DGMF_OK;
}

}  // namespace

}  // namespace dgmf

using namespace dgmf;

extern "C" {

dgmf_status dgmf_cg_workspace_bytes(dgmf_op op, const dgmf_cg_params* params, size_t* bytes) {
  dgmf_status e = validate(op, params);
  if (e) return e;
  if (!bytes) return fail(DGMF_INVALID, "cg_workspace_bytes: null output");
  const size_t es = params->precond_dtype == DGMF_F32 ? 4 : 8;
  *bytes = make_layout(op->mesh->ndofs, nparts_for(op), params->precond == 1, es).total;
  return DGMF_OK;
}

dgmf_status dgmf_cg_solve(dgmf_op op, const double* b, double* x, const dgmf_cg_params* params, void* workspace,
                          size_t workspace_bytes, hipStream_t stream, dgmf_cg_result* out) {
  dgmf_status e = validate(op, params);
  if (e) return e;
  if (!b || !x || !workspace || !out) return fail(DGMF_INVALID, "cg_solve: null argument");
  if (reinterpret_cast<uintptr_t>(b) % 8 || reinterpret_cast<uintptr_t>(x) % 8 ||
      reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(DGMF_INVALID, "cg_solve: misaligned argument (vectors 8 B, workspace 256 B)");
  const int64_t N = op->mesh->ndofs;
  const bool cheb = params->precond == 1;
  const size_t es = params->precond_dtype == DGMF_F32 ? 4 : 8;
  Layout L = make_layout(N, nparts_for(op), cheb, es);
  if (workspace_bytes < L.total)
    return fail(DGMF_INVALID, "cg_solve: workspace of %zu bytes, need %zu", workspace_bytes, L.total);
  {
    const char* wb = static_cast<const char*>(workspace);
    const char* xb = reinterpret_cast<const char*>(x);
    const char* bb = reinterpret_cast<const char*>(b);
    if ((xb < wb + L.total && wb < xb + 8 * N) || (bb < wb + L.total && wb < bb + 8 * N) ||
        (xb < bb + 8 * N && bb < xb + 8 * N))
      return fail(DGMF_INVALID, "cg_solve: b, x and workspace must not overlap");
  }
  int prev_dev = -1;
  (void)hipGetDevice(&prev_dev);
  if (prev_dev != op->mesh->device) DGMF_HIP_TRY(hipSetDevice(op->mesh->device));
  struct Restore {
    int d;
    ~Restore() { if (d >= 0) (void)hipSetDevice(d); }
  } restore{prev_dev != op->mesh->device ? prev_dev : -1};

  std::memset(out, 0, sizeof(*out));
  out->status = DGMF_OK;
  e = cg_run(op, b, x, params, static_cast<char*>(workspace), L, stream, out);
  if (e != DGMF_OK) {
    (void)hipStreamSynchronize(stream);
    out->status = e;
  }
  return e;
}

}  // extern "C"

namespace dgmf {
namespace {

// Workspace of dgmf_cg_solve_noalloc: a static array of the code object, so
// every device the library runs on holds one copy from module load to the
// end of the process.  Host code never uses the name `scratch` as an address
// (on the host it is a stand-in, not device memory): it asks the runtime for
// the current device's address once per device and passes that pointer on.
static __device__ __align__(256) char scratch[DGMF_CG_NOALLOC_MAX_BYTES];

struct NoAllocSlot {
  std::mutex lock;       // held for a whole (synchronous) solve on this device
  char* ptr = nullptr;   // device address of this device's copy of scratch
};

NoAllocSlot* noalloc_slot(int dev) {
  static std::mutex table_lock;
  static std::vector<std::unique_ptr<NoAllocSlot>> slots;
  std::lock_guard<std::mutex> g(table_lock);
  if (dev >= static_cast<int>(slots.size())) slots.resize(dev + 1);
  if (!slots[dev]) slots[dev] = std::make_unique<NoAllocSlot>();
  return slots[dev].get();
}

}  // namespace
}  // namespace dgmf

extern "C" {

dgmf_status dgmf_cg_solve_noalloc(dgmf_op op, const double* b, double* x, const dgmf_cg_params* params,
                                  hipStream_t stream, dgmf_cg_result* out) {
  dgmf_status e = validate(op, params);
  if (e) return e;
  if (params->precond == 2)
    return fail(DGMF_UNSUPPORTED, "cg_solve_noalloc: the multigrid hierarchy allocates; use precond 0, 1 or 3");
  if (!b || !x || !out) return fail(DGMF_INVALID, "cg_solve_noalloc: null argument");
  if (reinterpret_cast<uintptr_t>(b) % 8 || reinterpret_cast<uintptr_t>(x) % 8)
    return fail(DGMF_INVALID, "cg_solve_noalloc: misaligned vector (8 B)");
  const int64_t N = op->mesh->ndofs;
  const size_t es = params->precond_dtype == DGMF_F32 ? 4 : 8;
  Layout L = make_layout(N, nparts_for(op), params->precond == 1, es);
  if (L.total > DGMF_CG_NOALLOC_MAX_BYTES)
    return fail(DGMF_INVALID, "cg_solve_noalloc: %lld DoF need %zu bytes of workspace, more than the %zu bytes "
                "of the static buffer; use dgmf_cg_solve with a caller workspace",
                static_cast<long long>(N), L.total, static_cast<size_t>(DGMF_CG_NOALLOC_MAX_BYTES));
  {
    const char* xb = reinterpret_cast<const char*>(x);
    const char* bb = reinterpret_cast<const char*>(b);
    if (xb < bb + 8 * N && bb < xb + 8 * N) return fail(DGMF_INVALID, "cg_solve_noalloc: b and x overlap");
  }
  const int dev = op->mesh->device;
  int prev_dev = -1;
  (void)hipGetDevice(&prev_dev);
  if (prev_dev != dev) DGMF_HIP_TRY(hipSetDevice(dev));
  struct Restore {
    int d;
    ~Restore() { if (d >= 0) (void)hipSetDevice(d); }
  } restore{prev_dev != dev ? prev_dev : -1};
  NoAllocSlot* slot = noalloc_slot(dev);
  std::lock_guard<std::mutex> g(slot->lock);
  if (!slot->ptr) {
    // first call on this device, with the device current: its copy's address
    void* p = nullptr;
    const hipError_t he = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (he != hipSuccess || !p)
      return fail(DGMF_HIP_ERROR, "cg_solve_noalloc: hipGetSymbolAddress of the static buffer failed: %s",
                  hipGetErrorString(he));
    slot->ptr = static_cast<char*>(p);
  }
  {
    const char* wb = slot->ptr;
    const char* xb = reinterpret_cast<const char*>(x);
    const char* bb = reinterpret_cast<const char*>(b);
    if ((xb < wb + L.total && wb < xb + 8 * N) || (bb < wb + L.total && wb < bb + 8 * N))
      return fail(DGMF_INVALID, "cg_solve_noalloc: b or x lies in the library's static buffer");
  }
  std::memset(out, 0, sizeof(*out));
  out->status = DGMF_OK;
  // every value of the workspace is written before it is read (state by a
  // copy, partials and vectors by the kernels), so the previous call's
  // contents need no clearing
  e = cg_run(op, b, x, params, slot->ptr, L, stream, out);
  if (e != DGMF_OK) {
    (void)hipStreamSynchronize(stream);
    out->status = e;
  }
  return e;
}

dgmf_status dgmf_precond_apply(dgmf_op op, const dgmf_cg_params* params, const double* r, double* z,
                               hipStream_t stream) {
  dgmf_status e = validate(op, params);
  if (e) return e;
  if (params->precond != 2) return fail(DGMF_UNSUPPORTED, "precond_apply: only precond = 2 (multigrid) is exposed");
  if (!r || !z) return fail(DGMF_INVALID, "precond_apply: null vector");
  if (reinterpret_cast<uintptr_t>(r) % 8 || reinterpret_cast<uintptr_t>(z) % 8)
    return fail(DGMF_INVALID, "precond_apply: misaligned vector");
  const int64_t N = op->mesh->ndofs;
  {
    const char* a = reinterpret_cast<const char*>(r);
    const char* b = reinterpret_cast<const char*>(z);
    if (a < b + 8 * N && b < a + 8 * N) return fail(DGMF_INVALID, "precond_apply: r and z overlap");
  }
  int prev_dev = -1;
  (void)hipGetDevice(&prev_dev);
  if (prev_dev != op->mesh->device) DGMF_HIP_TRY(hipSetDevice(op->mesh->device));
  struct Restore {
    int d;
    ~Restore() { if (d >= 0) (void)hipSetDevice(d); }
  } restore{prev_dev != op->mesh->device ? prev_dev : -1};
  if ((e = mg_ensure(op, *params, stream))) return e;
  MgLevel& a = op->mgh->lv[0];
  if (params->precond_dtype == DGMF_F32) {
    if ((e = launch_mg_cast_in<float>(r, a.v<float>(0), N, nullptr, stream))) return e;
    if ((e = vcycle_run<float>(*op->mgh, nullptr, params->mg_graph != 0, stream))) return e;
    return launch_mg_cast_out<float>(a.v<float>(a.xout), z, N, stream);
  }
  if ((e = launch_mg_cast_in<double>(r, a.v<double>(0), N, nullptr, stream))) return e;
  if ((e = vcycle_run<double>(*op->mgh, nullptr, params->mg_graph != 0, stream))) return e;
  return launch_mg_cast_out<double>(a.v<double>(a.xout), z, N, stream);
}

dgmf_status dgmf_precond_info(dgmf_op op, int* levels, double* lambdas, int* coarse_degree, double* coarse_interval) {
  if (!op || op->kind != 1) return fail(DGMF_INVALID, "precond_info: not an SIPG operator");
  if (!op->mgh) return fail(DGMF_INVALID, "precond_info: no multigrid hierarchy has been built on this operator");
  const auto& lv = op->mgh->lv;
  const int L = static_cast<int>(lv.size());
  if (levels) *levels = L;
  if (lambdas)
    for (int l = 0; l < L; ++l) lambdas[l] = lv[l].lambda;
  if (coarse_degree) *coarse_degree = lv[L - 1].m;
  if (coarse_interval) {
    coarse_interval[0] = lv[L - 1].lo;
    coarse_interval[1] = lv[L - 1].hi;
  }
  return DGMF_OK;
}

}  // extern "C"
