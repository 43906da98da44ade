// Preconditioned CG for the implicit viscous step in its symmetric-gradient
// form (Sec. 3.2, implicit viscous step with s = 1 and F^nu(u) = 2 nu eps(u);
// Sec. 5.1: the viscous step is solved by CG).  The operator is
// H_eps = mu M + (scalar SIPG operator on every component) + nu C(u) (the
// component coupling of eps.hip); the preconditioner is the inverse diagonal
// of the scalar part, the same on the three components, or the inverse mass
// matrix on every component (the paper's viscous preconditioner, Sec. 5.1).
// Plain PCG in fp64
// with every scalar on the device: vector kernels write per-block partial
// sums, one single-block kernel adds them in a fixed order and advances
// alpha / beta, and a device status word idles the remaining kernels of a
// batch once the solve has stopped, so the host reads the state only every
// check_every iterations.
#include <chrono>
#include <cmath>
#include <cstring>

#include "internal.h"

namespace dgmf {
namespace {

// makes the operator's device current for the call, restores the caller's
struct DevScope {
  int prev = -1;
  explicit DevScope(int dev) {
    if (hipGetDevice(&prev) == hipSuccess && prev != dev) (void)hipSetDevice(dev);
  }
  ~DevScope() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

constexpr int kBlocks = 1024, kThreads = 256;
constexpr int V_RUNNING = 0, V_CONVERGED = 1;

struct VState {
  double rz, rr, bb, alpha, beta, tol2;
  int iter, max_iter, status, pad;
};

struct VLayout {
  size_t state, part, r, z, p, q, dinv, total;
};

VLayout vlayout(int64_t N) {
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  VLayout L{};
  size_t o = 0;
  L.state = o;
  o += up(sizeof(VState));
  L.part = o;
  o += up(3 * kBlocks * sizeof(double));
  const size_t v3 = up(static_cast<size_t>(3 * N) * sizeof(double)), v1 = up(static_cast<size_t>(N) * sizeof(double));
  L.r = o;
  o += v3;
  L.z = o;
  o += v3;
  L.p = o;
  o += v3;
  L.q = o;
  o += v3;
  L.dinv = o;
  o += v1;
  L.total = o;
  return L;
}

// sum of v over the block, the same order on every launch
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int o = kThreads / 2; o > 0; o >>= 1) {
    if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ void __launch_bounds__(kThreads) k_v_recip(const double* __restrict__ d, double* __restrict__ di,
                                                      int64_t n) {
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    di[i] = 1.0 / d[i];
}

// r = b - q, z = dinv r; partials <r,z>, <r,r>, <b,b>
__global__ void __launch_bounds__(kThreads) k_v_init(const double* __restrict__ b, const double* __restrict__ q,
                                                     double* __restrict__ r, double* __restrict__ z,
                                                     const double* __restrict__ dinv, int64_t N, double* part) {
  __shared__ double sh[kThreads];
  double rz = 0, rr = 0, bb = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < 3 * N;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    const double bi = b[i], ri = bi - q[i], zi = dinv[i % N] * ri;
    r[i] = ri;
    z[i] = zi;
    rz = fma(ri, zi, rz);
    rr = fma(ri, ri, rr);
    bb = fma(bi, bi, bb);
  }
  rz = block_sum(rz, sh);
  rr = block_sum(rr, sh);
  bb = block_sum(bb, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rz;
    part[kBlocks + blockIdx.x] = rr;
    part[2 * kBlocks + blockIdx.x] = bb;
  }
}

// partial <p, q>
__global__ void __launch_bounds__(kThreads) k_v_pq(const double* __restrict__ p, const double* __restrict__ q,
                                                   int64_t n3, double* part, const VState* st) {
  if (st->status != V_RUNNING) return;
  __shared__ double sh[kThreads];
  double s = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n3;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    s = fma(p[i], q[i], s);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// x += alpha p, r -= alpha q, z = dinv r; partials <r,r>, <r,z>
__global__ void __launch_bounds__(kThreads) k_v_update(double* __restrict__ x, double* __restrict__ r,
                                                       const double* __restrict__ p, const double* __restrict__ q,
                                                       double* __restrict__ z, const double* __restrict__ dinv,
                                                       int64_t N, double* part, const VState* st) {
  if (st->status != V_RUNNING) return;
  __shared__ double sh[kThreads];
  const double a = st->alpha;
  double rr = 0, rz = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < 3 * N;
       i += static_cast<int64_t>(gridDim.x) * kThreads) {
    x[i] = fma(a, p[i], x[i]);
    const double ri = fma(-a, q[i], r[i]), zi = dinv[i % N] * ri;
    r[i] = ri;
    z[i] = zi;
    rr = fma(ri, ri, rr);
    rz = fma(ri, zi, rz);
  }
  rr = block_sum(rr, sh);
  rz = block_sum(rz, sh);
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rr;
    part[kBlocks + blockIdx.x] = rz;
  }
}

// partials <r, z> into part[slot * kBlocks + block] (z from the inverse mass)
__global__ void __launch_bounds__(kThreads) k_v_rz(const double* __restrict__ r, const double* __restrict__ z,
                                                   int64_t n3, double* part, int slot, const VState* st, int always) {
  if (!always && st->status != V_RUNNING) return;
  __shared__ double sh[kThreads];
  double s = 0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n3;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    s = fma(r[i], z[i], s);
  s = block_sum(s, sh);
  if (threadIdx.x == 0) part[slot * kBlocks + blockIdx.x] = s;
}

// p = z + beta p (first: p = z)
__global__ void __launch_bounds__(kThreads) k_v_pupdate(double* __restrict__ p, const double* __restrict__ z,
                                                        int64_t n3, const VState* st, int first) {
  if (!first && st->status != V_RUNNING) return;
  const double b = first ? 0.0 : st->beta;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n3;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    p[i] = first ? z[i] : fma(b, p[i], z[i]);
}

enum { VM_INIT = 0, VM_ALPHA = 1, VM_BETA = 2 };

// one workgroup: fixed-order sums of the partials, then the scalar recurrences
__global__ void __launch_bounds__(kThreads) k_v_scalar(VState* st, const double* part, int mode) {
  if (mode != VM_INIT && st->status != V_RUNNING) return;
  __shared__ double sh[kThreads];
  double s[3] = {0, 0, 0};
  const int nsum = mode == VM_INIT ? 3 : (mode == VM_ALPHA ? 1 : 2);
  for (int k = 0; k < nsum; ++k) {
    double a = 0;
    for (int i = threadIdx.x; i < kBlocks; i += kThreads) a += part[k * kBlocks + i];
    s[k] = block_sum(a, sh);
  }
  if (threadIdx.x != 0) return;
  if (mode == VM_INIT) {
    st->rz = s[0];
    st->rr = s[1];
    st->bb = s[2];
    st->iter = 0;
    if (!isfinite(s[0]) || !isfinite(s[1])) st->status = DGMF_NONFINITE;
    else if (s[1] <= st->tol2 * s[2]) st->status = V_CONVERGED;
    else if (st->max_iter <= 0) st->status = DGMF_NOT_CONVERGED;
    else st->status = V_RUNNING;
  } else if (mode == VM_ALPHA) {
    const double pq = s[0];
    if (!isfinite(pq)) st->status = DGMF_NONFINITE;
    else if (!(pq > 0)) st->status = DGMF_BREAKDOWN;
    else st->alpha = st->rz / pq;
  } else {
    const double rr = s[0], rz = s[1];
    st->rr = rr;
    st->iter += 1;
    if (!isfinite(rr) || !isfinite(rz)) st->status = DGMF_NONFINITE;
    else if (rr <= st->tol2 * st->bb) st->status = V_CONVERGED;
    else if (st->iter >= st->max_iter) st->status = DGMF_NOT_CONVERGED;
    else {
      st->beta = rz / st->rz;
      st->rz = rz;
    }
  }
}

dgmf_status apply_eps(dgmf_op op, const double* u, double* out, hipStream_t s) {
  return viscous_apply_any(op, u, out, s);
}

// z = M^{-1} r on the three components (the point-weight form on curved cells)
dgmf_status inv_mass3(dgmf_op op, const double* r, double* z, hipStream_t s) {
  const dgmf_mesh m = op->mesh;
  if (m->desc.curve_amp != 0.0)
    return launch_point_mass<double>(m->tab.n, static_cast<const double*>(m->pmt64.p), m->mg64.cm, r, z, m->ncells,
                                     3, true, s);
  return launch_block_mass<double>(m->tab.n, m->g64, 1.0 / std::fabs(m->shear.det),
                                   static_cast<const double*>(m->minv64.p), r, z, m->ncells, 3, true, s);
}

dgmf_status vcheck(dgmf_op op) {
  if (!op || op->kind != 1) return fail(DGMF_INVALID, "viscous_cg: not an SIPG operator");
  const dgmf_mesh m = op->mesh;
  if (m->shear.on) return fail(DGMF_UNSUPPORTED, "viscous_cg: sheared meshes are not supported");
  return DGMF_OK;
}

}  // namespace

}  // namespace dgmf

using namespace dgmf;

extern "C" {

dgmf_status dgmf_viscous_cg_workspace_bytes(dgmf_op op, size_t* bytes) {
  if (dgmf_status e = vcheck(op)) return e;
  if (!bytes) return fail(DGMF_INVALID, "viscous_cg_workspace_bytes: null argument");
  *bytes = vlayout(op->mesh->ndofs).total;
  return DGMF_OK;
}

dgmf_status dgmf_viscous_cg_solve(dgmf_op op, const double* b, double* x, const dgmf_cg_params* params,
                                  void* workspace, size_t workspace_bytes, hipStream_t stream, dgmf_cg_result* out) {
  if (dgmf_status e = vcheck(op)) return e;
  if (!b || !x || !params || !workspace || !out) return fail(DGMF_INVALID, "viscous_cg: null argument");
  if (params->precond != 0 && params->precond != 3)
    return fail(DGMF_UNSUPPORTED, "viscous_cg: preconditioner 0 (Jacobi) or 3 (inverse mass)");
  const bool mass = params->precond == 3;
  if (!(params->rtol >= 0) || !std::isfinite(params->rtol) || params->max_iter < 0 || params->check_every < 0)
    return fail(DGMF_INVALID, "viscous_cg: rtol must be finite and >= 0, max_iter and check_every >= 0");
  if (reinterpret_cast<uintptr_t>(b) % 8 || reinterpret_cast<uintptr_t>(x) % 8 ||
      reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(DGMF_INVALID, "viscous_cg: misaligned argument (vectors 8 B, workspace 256 B)");
  const int64_t N = op->mesh->ndofs;
  const VLayout L = vlayout(N);
  if (workspace_bytes < L.total)
    return fail(DGMF_INVALID, "viscous_cg: workspace of %zu bytes, need %zu", workspace_bytes, L.total);
  {
    const char* wb = static_cast<const char*>(workspace);
    const char* xb = reinterpret_cast<const char*>(x);
    const char* bb = reinterpret_cast<const char*>(b);
    const int64_t vb = 24 * N;
    if ((xb < wb + L.total && wb < xb + vb) || (bb < wb + L.total && wb < bb + vb) || (xb < bb + vb && bb < xb + vb))
      return fail(DGMF_INVALID, "viscous_cg: b, x and workspace must not overlap");
  }
  DevScope dev(op->mesh->device);
  std::memset(out, 0, sizeof(*out));
  // every non-OK return below leaves out->status equal to it and the stream drained
  auto run = [&]() -> dgmf_status {
    char* ws = static_cast<char*>(workspace);
    VState* st = reinterpret_cast<VState*>(ws + L.state);
    double* part = reinterpret_cast<double*>(ws + L.part);
    double* r = reinterpret_cast<double*>(ws + L.r);
    double* z = reinterpret_cast<double*>(ws + L.z);
    double* p = reinterpret_cast<double*>(ws + L.p);
    double* q = reinterpret_cast<double*>(ws + L.q);
    double* dinv = reinterpret_cast<double*>(ws + L.dinv);
    const dim3 G(kBlocks), B(kThreads);
    dgmf_status e;
    auto t0 = std::chrono::steady_clock::now();
    VState init{};
    init.tol2 = params->rtol * params->rtol;
    init.max_iter = params->max_iter;
    DGMF_HIP_TRY(hipMemcpyAsync(st, &init, sizeof(init), hipMemcpyHostToDevice, stream));
    hipLaunchKernelGGL(k_v_recip, G, B, 0, stream, static_cast<const double*>(op->diag64.p), dinv, N);
    DGMF_LAUNCH_CHECK("k_v_recip");
    if ((e = apply_eps(op, x, q, stream))) return e;
    hipLaunchKernelGGL(k_v_init, G, B, 0, stream, b, q, r, z, dinv, N, part);
    DGMF_LAUNCH_CHECK("k_v_init");
    if (mass) {   // z = M^{-1} r replaces the diagonal scaling, and <r, z> with it
      if ((e = inv_mass3(op, r, z, stream))) return e;
      hipLaunchKernelGGL(k_v_rz, G, B, 0, stream, r, z, 3 * N, part, 0, st, 1);
      DGMF_LAUNCH_CHECK("k_v_rz");
    }
    hipLaunchKernelGGL(k_v_scalar, dim3(1), B, 0, stream, st, part, static_cast<int>(VM_INIT));
    DGMF_LAUNCH_CHECK("k_v_scalar");
    hipLaunchKernelGGL(k_v_pupdate, G, B, 0, stream, p, z, 3 * N, st, 1);
    DGMF_LAUNCH_CHECK("k_v_pupdate");
    VState h{};
    DGMF_HIP_TRY(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, stream));
    DGMF_HIP_TRY(hipStreamSynchronize(stream));
    auto t1 = std::chrono::steady_clock::now();
    const int batch = params->check_every > 0 ? params->check_every : 1;
    while (h.status == V_RUNNING) {
      for (int k = 0; k < batch; ++k) {
        if ((e = apply_eps(op, p, q, stream))) return e;
        hipLaunchKernelGGL(k_v_pq, G, B, 0, stream, p, q, 3 * N, part, st);
        DGMF_LAUNCH_CHECK("k_v_pq");
        hipLaunchKernelGGL(k_v_scalar, dim3(1), B, 0, stream, st, part, static_cast<int>(VM_ALPHA));
        DGMF_LAUNCH_CHECK("k_v_scalar");
        hipLaunchKernelGGL(k_v_update, G, B, 0, stream, x, r, p, q, z, dinv, N, part, st);
        DGMF_LAUNCH_CHECK("k_v_update");
        if (mass) {
          if ((e = inv_mass3(op, r, z, stream))) return e;
          hipLaunchKernelGGL(k_v_rz, G, B, 0, stream, r, z, 3 * N, part, 1, st, 0);
          DGMF_LAUNCH_CHECK("k_v_rz");
        }
        hipLaunchKernelGGL(k_v_scalar, dim3(1), B, 0, stream, st, part, static_cast<int>(VM_BETA));
        DGMF_LAUNCH_CHECK("k_v_scalar");
        hipLaunchKernelGGL(k_v_pupdate, G, B, 0, stream, p, z, 3 * N, st, 0);
        DGMF_LAUNCH_CHECK("k_v_pupdate");
      }
      DGMF_HIP_TRY(hipMemcpyAsync(&h, st, sizeof(h), hipMemcpyDeviceToHost, stream));
      DGMF_HIP_TRY(hipStreamSynchronize(stream));
    }
    auto t2 = std::chrono::steady_clock::now();
    out->iterations = h.iter;
    out->rel_residual = h.bb > 0 ? std::sqrt(h.rr / h.bb) : 0.0;
    out->status = h.status == V_CONVERGED ? DGMF_OK : h.status;
    out->setup_s = std::chrono::duration<double>(t1 - t0).count();
    out->solve_s = std::chrono::duration<double>(t2 - t1).count();
    if (out->status != DGMF_OK)
      return fail(static_cast<dgmf_status>(out->status), "viscous_cg: status %d after %d iterations (rel. residual %g)",
                  out->status, out->iterations, out->rel_residual);
    return DGMF_OK;
  };
  const dgmf_status e = run();
  if (e != DGMF_OK) {
    (void)hipStreamSynchronize(stream);
    out->status = e;
  }
  return e;
}

}  // extern "C"
