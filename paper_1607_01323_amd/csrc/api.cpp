// C-ABI entry points of libdgmf: handles, validation, launches.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <type_traits>

#include "internal.h"

namespace dgmf {

namespace {
thread_local std::string g_last_error;

struct DeviceGuard {
  int prev = -1;
  bool ok = true;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
    if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};
}  // namespace

dgmf_status fail(dgmf_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return st;
}

void clear_error() { g_last_error.clear(); }

const char* last_error_cstr() { return g_last_error.c_str(); }

dgmf_status DevBuf::alloc(size_t nbytes) {
  release();
  if (nbytes == 0) return DGMF_OK;
  hipError_t e = hipMalloc(&p, nbytes);
  if (e != hipSuccess) {
    p = nullptr;
    return fail(e == hipErrorOutOfMemory ? DGMF_OOM : DGMF_HIP_ERROR, "hipMalloc(%zu) failed: %s", nbytes,
                hipGetErrorString(e));
  }
  bytes = nbytes;
  return DGMF_OK;
}

dgmf_status DevBuf::upload(const void* host, size_t nbytes) {
  dgmf_status st = alloc(nbytes);
  if (st != DGMF_OK) return st;
  DGMF_HIP_TRY(hipMemcpy(p, host, nbytes, hipMemcpyHostToDevice));
  return DGMF_OK;
}

void DevBuf::release() {
  if (p) (void)hipFree(p);
  p = nullptr;
  bytes = 0;
}

// Per-direction geometry arrays (x0, h, 1/h, tp) of a box mesh, contiguous.
// bit 2d+s set: boundary side (d, s) is homogeneous Neumann (stored normalised: 0 in periodic directions)
static int neumann_mask(const dgmf_box_desc& d) {
  int mask = 0;
  for (int f = 0; f < 6; ++f)
    if (d.neumann[f] && !d.periodic[f / 2]) mask |= 1 << f;
  return mask;
}

template <typename T>
static dgmf_status upload_geometry(dgmf_mesh m, DevBuf& buf, CartGeom<T>& g) {
  const int nd[3] = {m->desc.nx, m->desc.ny, m->desc.nz};
  std::vector<T> host;
  size_t off[3];
  for (int d = 0; d < 3; ++d) {
    off[d] = host.size();
    const auto& v = m->verts[d];
    for (int c = 0; c < nd[d]; ++c) host.push_back(static_cast<T>(v[c]));
    for (int c = 0; c < nd[d]; ++c) host.push_back(static_cast<T>(v[c + 1] - v[c]));
    for (int c = 0; c < nd[d]; ++c) host.push_back(static_cast<T>(1.0 / (v[c + 1] - v[c])));
    for (int c = 0; c < nd[d]; ++c) {
      double w = 1.0;   // two interior faces, half of each
      if (!m->desc.periodic[d]) {
        if (nd[d] == 1) w = 2.0;
        else if (c == 0 || c == nd[d] - 1) w = 1.5;
      }
      host.push_back(static_cast<T>(w / (v[c + 1] - v[c])));
    }
  }
  dgmf_status st = buf.upload(host.data(), host.size() * sizeof(T));
  if (st != DGMF_OK) return st;
  const T* base = static_cast<const T*>(buf.p);
  g.nx = nd[0];
  g.ny = nd[1];
  g.nz = nd[2];
  g.neu = neumann_mask(m->desc);
  for (int d = 0; d < 3; ++d) {
    g.per[d] = m->desc.periodic[d] ? 1 : 0;
    g.x0[d] = base + off[d];
    g.h[d] = base + off[d] + nd[d];
    g.hinv[d] = base + off[d] + 2 * nd[d];
    g.tp[d] = base + off[d] + 3 * nd[d];
  }
  return DGMF_OK;
}

template <typename T>
static dgmf_status upload_tables(const Tables1D& t, DevBuf& buf, const std::vector<double>* xhat = nullptr) {
  TabLayout L{t.n, t.nq};
  std::vector<T> h(L.size(), T(0));
  if (xhat)
    for (int i = 0; i < t.n * t.n; ++i) h[L.xhat() + i] = static_cast<T>((*xhat)[i]);
  for (int i = 0; i < t.n * t.n; ++i) {
    h[L.mhat() + i] = static_cast<T>(t.Mhat[i]);
    h[L.khat() + i] = static_cast<T>(t.Khat[i]);
  }
  for (int i = 0; i < t.n; ++i) {
    h[L.g0() + i] = static_cast<T>(t.g0[i]);
    h[L.g1() + i] = static_cast<T>(t.g1[i]);
    h[L.nodes() + i] = static_cast<T>(t.nodes[i]);
  }
  for (int i = 0; i < t.nq * t.n; ++i) h[L.S() + i] = static_cast<T>(t.S[i]);
  for (int q = 0; q < t.nq; ++q) {
    h[L.wq() + q] = static_cast<T>(t.wq[q]);
    h[L.xq() + q] = static_cast<T>(t.xq[q]);
  }
  if (t.nq == t.n) {
    // Mhat^{-1} by Gauss-Jordan elimination with partial pivoting in long double
    const int n = t.n;
    std::vector<long double> a(n * 2 * n, 0.0L);
    for (int i = 0; i < n; ++i) {
      for (int j = 0; j < n; ++j) a[i * 2 * n + j] = t.Mhat[i * n + j];
      a[i * 2 * n + n + i] = 1.0L;
    }
    for (int c = 0; c < n; ++c) {
      int piv = c;
      for (int r = c + 1; r < n; ++r)
        if (std::fabs(static_cast<double>(a[r * 2 * n + c])) > std::fabs(static_cast<double>(a[piv * 2 * n + c]))) piv = r;
      for (int j = 0; j < 2 * n; ++j) std::swap(a[c * 2 * n + j], a[piv * 2 * n + j]);
      const long double d = a[c * 2 * n + c];
      for (int j = 0; j < 2 * n; ++j) a[c * 2 * n + j] /= d;
      for (int r = 0; r < n; ++r)
        if (r != c) {
          const long double f = a[r * 2 * n + c];
          for (int j = 0; j < 2 * n; ++j) a[r * 2 * n + j] -= f * a[c * 2 * n + j];
        }
    }
    auto minv = [&](int i, int j) { return a[i * 2 * n + n + j]; };
    for (int i = 0; i < n; ++i) {
      long double g0 = 0, g1 = 0;
      for (int j = 0; j < n; ++j) {
        long double kk = 0;
        for (int m = 0; m < n; ++m) kk += minv(i, m) * t.Khat[m * n + j];
        h[L.ktil() + i * n + j] = static_cast<T>(kk);
        g0 += minv(i, j) * t.g0[j];
        g1 += minv(i, j) * t.g1[j];
      }
      h[L.g0t() + i] = static_cast<T>(g0);
      h[L.g1t() + i] = static_cast<T>(g1);
      h[L.e0t() + i] = static_cast<T>(minv(i, 0));
      h[L.e1t() + i] = static_cast<T>(minv(i, n - 1));
    }
  }
  return buf.upload(h.data(), h.size() * sizeof(T));
}

// Inverse of a small dense matrix by Gauss-Jordan elimination with partial
// pivoting in long double; false when singular.
static bool invert(int n, const double* a_in, std::vector<long double>& inv) {
  std::vector<long double> a(n * 2 * n, 0.0L);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) a[i * 2 * n + j] = a_in[i * n + j];
    a[i * 2 * n + n + i] = 1.0L;
  }
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(static_cast<double>(a[r * 2 * n + c])) > std::fabs(static_cast<double>(a[piv * 2 * n + c]))) piv = r;
    if (a[piv * 2 * n + c] == 0.0L) return false;
    for (int j = 0; j < 2 * n; ++j) std::swap(a[c * 2 * n + j], a[piv * 2 * n + j]);
    const long double d = a[c * 2 * n + c];
    for (int j = 0; j < 2 * n; ++j) a[c * 2 * n + j] /= d;
    for (int r = 0; r < n; ++r)
      if (r != c) {
        const long double f = a[r * 2 * n + c];
        for (int j = 0; j < 2 * n; ++j) a[r * 2 * n + j] -= f * a[c * 2 * n + j];
      }
  }
  inv.assign(n * n, 0.0L);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) inv[i * n + j] = a[i * 2 * n + n + j];
  return true;
}

bool inverse_mass_1d(const Tables1D& t, std::vector<double>& out) {
  const int n = t.n;
  if (t.nq != n) return false;
  std::vector<long double> sinv;
  if (!invert(n, t.S.data(), sinv)) return false;
  out.assign(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      long double a = 0;
      for (int q = 0; q < n; ++q) a += sinv[i * n + q] * sinv[j * n + q] / static_cast<long double>(t.wq[q]);
      out[i * n + j] = static_cast<double>(a);
    }
  return true;
}

// Quadrature-point metric of a lattice mesh: tables S, D, Dg = D S^{-1},
// l'(0), l'(1), w; cell and face geometry filled on the device in fp64, then
// copied to fp32.
static dgmf_status setup_metric(dgmf_mesh m) {
  const int n = m->tab.n;
  const Tables1D& t = m->tab;
  const int nd[3] = {m->desc.nx, m->desc.ny, m->desc.nz};
  std::vector<long double> sinv;
  if (!invert(n, t.S.data(), sinv)) return fail(DGMF_INVALID, "mesh_create: singular interpolation matrix");
  std::vector<double> tab(metric_tab_size(n), 0.0);
  for (int i = 0; i < n * n; ++i) {
    tab[i] = t.S[i];
    tab[n * n + i] = t.D[i];
  }
  for (int q = 0; q < n; ++q)
    for (int j = 0; j < n; ++j) {
      long double a = 0;
      for (int m2 = 0; m2 < n; ++m2) a += static_cast<long double>(t.D[q * n + m2]) * sinv[m2 * n + j];
      tab[2 * n * n + q * n + j] = static_cast<double>(a);
    }
  for (int i = 0; i < n; ++i) {
    tab[3 * n * n + i] = t.g0[i];
    tab[3 * n * n + n + i] = t.g1[i];
    tab[3 * n * n + 2 * n + i] = t.wq[i];
    // Lagrange basis through the Gauss points, at 0 and at 1
    long double e0 = 1.0L, e1 = 1.0L;
    for (int k = 0; k < n; ++k)
      if (k != i) {
        const long double den = static_cast<long double>(t.xq[i]) - t.xq[k];
        e0 *= (0.0L - t.xq[k]) / den;
        e1 *= (1.0L - t.xq[k]) / den;
      }
    tab[3 * n * n + 3 * n + i] = static_cast<double>(e0);
    tab[3 * n * n + 4 * n + i] = static_cast<double>(e1);
  }
  std::vector<float> tab32(tab.begin(), tab.end());
  dgmf_status st = m->mtab64.upload(tab.data(), tab.size() * sizeof(double));
  if (st == DGMF_OK) st = m->mtab32.upload(tab32.data(), tab32.size() * sizeof(float));
  if (st != DGMF_OK) return st;

  const int64_t nc = m->ncells, n2 = n * n, n3 = n2 * n;
  int64_t nlow = 0;
  int lbase[3] = {0, 0, 0};
  for (int d = 0; d < 3; ++d) {
    lbase[d] = static_cast<int>(nlow);
    if (!m->desc.periodic[d]) nlow += static_cast<int64_t>(nd[0]) * nd[1] * nd[2] / nd[d];
  }
  const int64_t o_cm = 0, o_fm = o_cm + nc * 7 * n3, o_ft = o_fm + nc * 21 * n2, o_lm = o_ft + nc * 3,
                o_lt = o_lm + nlow * 7 * n2, total = o_lt + nlow;
  if ((st = m->met64.alloc(static_cast<size_t>(total) * 8))) return st;
  if ((st = m->met32.alloc(static_cast<size_t>(total) * 4))) return st;
  auto setg = [&](auto& g, auto* base, auto* tb) {
    g.nx = nd[0];
    g.ny = nd[1];
    g.nz = nd[2];
    g.neu = neumann_mask(m->desc);
    for (int d = 0; d < 3; ++d) {
      g.per[d] = m->desc.periodic[d] ? 1 : 0;
      g.lbase[d] = lbase[d];
    }
    g.cm = base + o_cm;
    g.fm = base + o_fm;
    g.ftau = base + o_ft;
    g.lm = base + o_lm;
    g.ltau = base + o_lt;
    g.tab = tb;
  };
  double* b64 = static_cast<double*>(m->met64.p);
  setg(m->mg64, static_cast<const double*>(b64), static_cast<const double*>(m->mtab64.p));
  setg(m->mg32, static_cast<const float*>(m->met32.p), static_cast<const float*>(m->mtab32.p));
  const double* x0[3] = {m->g64.x0[0], m->g64.x0[1], m->g64.x0[2]};
  const double* h[3] = {m->g64.h[0], m->g64.h[1], m->g64.h[2]};
  std::vector<long double> shinv;
  if (!invert(3, m->shear.m, shinv)) return fail(DGMF_INVALID, "mesh_create: singular shear");
  double shi[9];
  for (int i = 0; i < 9; ++i) shi[i] = static_cast<double>(shinv[i]);
  const double* wdev = static_cast<const double*>(m->mtab64.p) + 3 * n * n + 2 * n;
  if (m->desc.curve_amp != 0.0) {
    // GLL nodes, S, D (rows at the Gauss points), l(0), l(1), l'(0), l'(1), Gauss weights
    std::vector<double> ct(6 * n + 2 * n * n, 0.0);
    for (int i = 0; i < n; ++i) ct[i] = t.nodes[i];
    for (int i = 0; i < n * n; ++i) {
      ct[n + i] = t.S[i];
      ct[n + n * n + i] = t.D[i];
    }
    ct[n + 2 * n * n] = 1.0;
    ct[2 * n + 2 * n * n + n - 1] = 1.0;
    for (int i = 0; i < n; ++i) {
      ct[3 * n + 2 * n * n + i] = t.g0[i];
      ct[4 * n + 2 * n * n + i] = t.g1[i];
      ct[5 * n + 2 * n * n + i] = t.wq[i];
    }
    DevBuf ctab, taue;
    if ((st = ctab.upload(ct.data(), ct.size() * sizeof(double)))) return st;
    if ((st = taue.alloc(static_cast<size_t>(nc) * sizeof(double)))) return st;
    const double lo[3] = {0.0, m->desc.y0, 0.0};
    const double len[3] = {m->desc.lx, m->desc.ly, m->desc.lz};
    if ((st = launch_metric_fill_curved(n, m->mg64, x0, h, lo, len, m->desc.curve_amp,
                                        static_cast<const double*>(ctab.p), static_cast<double*>(taue.p),
                                        b64 + o_cm, b64 + o_fm, b64 + o_ft, b64 + o_lm, b64 + o_lt, nullptr)))
      return st;
    DGMF_HIP_TRY(hipStreamSynchronize(nullptr));   // the scratch buffers are released at return
  } else if ((st = launch_metric_fill(n, m->mg64, x0, h, shi, m->shear.det, wdev, b64 + o_cm, b64 + o_fm,
                                      b64 + o_ft, b64 + o_lm, b64 + o_lt, nullptr))) {
    return st;
  }
  if ((st = launch_to_f32(b64, static_cast<float*>(m->met32.p), total, nullptr))) return st;
  DGMF_HIP_TRY(hipStreamSynchronize(nullptr));
  return DGMF_OK;
}

// Line operators of a uniform, fully periodic mesh (layout UTab).  With
// Kt = Mhat^-1 Khat and the Mhat^-1 images g0t, g1t, e0t, e1t of l'(0),
// l'(1), e_0, e_{n-1}, one direction's contribution to
//   w = mu u + sum_d (nu/h_d) Mhat^-1 A_d u        (per unit cell volume V)
// is, with s = nu V / h_d, h = h_d and tau the face penalty,
//   w += s/h (Abar u) + s [ 1/2 ur_0/h g1t + (tau (u_{n-1} - ur_0) - 1/2 l'(0).ur/h) e1t
//                         - 1/2 ul_{n-1}/h g0t + (tau (u_0 - ul_{n-1}) + 1/2 l'(1).ul/h) e0t ],
//   Abar = Kt + 1/2 (g0t e_0^T - g1t e_{n-1}^T + e0t l'(0)^T - e1t l'(1)^T),
// the own-cell part of both face fluxes folded into Abar.  mu V is added to
// the diagonal of the z operator.
template <typename T>
static dgmf_status upload_uniform_tables(const Tables1D& t, const double h[3], double mu, double nu, double pen,
                                         DevBuf& buf) {
  const int n = t.n;
  UTab L{n};
  std::vector<long double> minv;
  if (!invert(n, t.Mhat.data(), minv)) return fail(DGMF_INVALID, "sipg_create: singular mass matrix");
  auto mv = [&](const std::vector<double>& v, int i) {
    long double a = 0;
    for (int m = 0; m < n; ++m) a += minv[i * n + m] * v[m];
    return a;
  };
  std::vector<long double> kt(n * n), g0t(n), g1t(n), e0t(n), e1t(n), abar(n * n);
  for (int i = 0; i < n; ++i) {
    for (int j = 0; j < n; ++j) {
      long double a = 0;
      for (int m = 0; m < n; ++m) a += minv[i * n + m] * t.Khat[m * n + j];
      kt[i * n + j] = a;
    }
    g0t[i] = mv(t.g0, i);
    g1t[i] = mv(t.g1, i);
    e0t[i] = minv[i * n];
    e1t[i] = minv[i * n + n - 1];
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      abar[i * n + j] = kt[i * n + j] +
                        0.5L * ((j == 0 ? g0t[i] : 0.0L) - (j == n - 1 ? g1t[i] : 0.0L) + e0t[i] * t.g0[j] -
                                e1t[i] * t.g1[j]);
  const long double V = static_cast<long double>(h[0]) * h[1] * h[2];
  const long double tau = pen * (1.0L / h[0] + 1.0L / h[1] + 1.0L / h[2]);
  std::vector<T> out(L.size(), T(0));
  for (int d = 0; d < 3; ++d) {
    const long double hi = 1.0L / h[d], s = nu * V * hi;
    for (int i = 0; i < n * n; ++i) out[L.A(d) + i] = static_cast<T>(s * hi * abar[i]);
    if (d == 2)
      for (int i = 0; i < n; ++i) out[L.A(d) + i * n + i] = static_cast<T>(s * hi * abar[i * n + i] + mu * V);
    for (int i = 0; i < n; ++i) {
      out[L.G1(d) + i] = static_cast<T>(0.5L * s * hi * g1t[i]);
      out[L.G0(d) + i] = static_cast<T>(-0.5L * s * hi * g0t[i]);
      out[L.g0s(d) + i] = static_cast<T>(-0.5L * s * hi * t.g0[i]);
      out[L.g1s(d) + i] = static_cast<T>(0.5L * s * hi * t.g1[i]);
    }
    out[L.c(d)] = static_cast<T>(s * tau);
  }
  for (int i = 0; i < n; ++i) {
    out[L.E1() + i] = static_cast<T>(e1t[i]);
    out[L.E0() + i] = static_cast<T>(e0t[i]);
  }
  for (int i = 0; i < n * n; ++i) out[L.Mh() + i] = static_cast<T>(t.Mhat[i]);
  return buf.upload(out.data(), out.size() * sizeof(T));
}

static bool aligned(const void* p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

static bool overlap(const void* a, const void* b, size_t bytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bytes && y < x + bytes;
}

// [a, a + abytes) and [b, b + bbytes) intersect
static bool overlap2(const void* a, size_t abytes, const void* b, size_t bbytes) {
  const char* x = static_cast<const char*>(a);
  const char* y = static_cast<const char*>(b);
  return x < y + bbytes && y < x + abytes;
}

}  // namespace dgmf

using namespace dgmf;

extern "C" {

const char* dgmf_last_error(void) { return last_error_cstr(); }

int dgmf_version(void) { return 100; }

dgmf_status dgmf_mesh_create(const dgmf_box_desc* desc, dgmf_mesh* out) {
  if (!desc || !out) return fail(DGMF_INVALID, "mesh_create: null argument");
  const dgmf_box_desc& d = *desc;
  if (d.degree < kMinDegree || d.degree > kMaxDegree)
    return fail(DGMF_INVALID, "mesh_create: degree %d outside %d..%d", d.degree, kMinDegree, kMaxDegree);
  if (d.nx < 1 || d.ny < 1 || d.nz < 1) return fail(DGMF_INVALID, "mesh_create: cell counts must be >= 1");
  if (!(d.lx > 0) || !(d.ly > 0) || !(d.lz > 0) || !std::isfinite(d.lx) || !std::isfinite(d.ly) ||
      !std::isfinite(d.lz) || !std::isfinite(d.y0))
    return fail(DGMF_INVALID, "mesh_create: lengths must be finite and > 0");
  if (!(d.y_tanh_gamma >= 0) || !std::isfinite(d.y_tanh_gamma))
    return fail(DGMF_INVALID, "mesh_create: y_tanh_gamma must be finite and >= 0");
  for (int f = 0; f < 6; ++f)
    if (d.neumann[f] != 0 && d.neumann[f] != 1) return fail(DGMF_INVALID, "mesh_create: neumann[%d] must be 0 or 1", f);
  Shear sh{{1, 0, 0, 0, 1, 0, 0, 0, 1}, 1.0, 0};
  {
    bool zero = true, ident = true;
    for (int i = 0; i < 9; ++i) {
      if (!std::isfinite(d.shear[i])) return fail(DGMF_INVALID, "mesh_create: shear entries must be finite");
      if (d.shear[i] != 0.0) zero = false;
      if (d.shear[i] != (i % 4 == 0 ? 1.0 : 0.0)) ident = false;
    }
    if (!zero && !ident) {
      for (int i = 0; i < 9; ++i) sh.m[i] = d.shear[i];
      const double* a = d.shear;
      sh.det = a[0] * (a[4] * a[8] - a[5] * a[7]) - a[1] * (a[3] * a[8] - a[5] * a[6]) +
               a[2] * (a[3] * a[7] - a[4] * a[6]);
      double nrm = 0.0;
      for (int i = 0; i < 9; ++i) nrm = std::max(nrm, std::fabs(a[i]));
      if (!(std::fabs(sh.det) > 1e-12 * nrm * nrm * nrm))
        return fail(DGMF_INVALID, "mesh_create: shear matrix is singular");
      sh.on = 1;
      if (!d.store_qp_metric)
        return fail(DGMF_INVALID, "mesh_create: a non-identity shear needs store_qp_metric = 1");
    }
  }
  if (!std::isfinite(d.curve_amp) || std::fabs(d.curve_amp) > 0.1)
    return fail(DGMF_INVALID, "mesh_create: curve_amp must be finite with |curve_amp| <= 0.1");
  if (d.curve_amp != 0.0) {
    if (!d.store_qp_metric) return fail(DGMF_INVALID, "mesh_create: curved cells need store_qp_metric = 1");
    if (sh.on) return fail(DGMF_INVALID, "mesh_create: curve_amp and a shear exclude each other");
  }
  if (d.store_qp_metric) {
    const int ndc[3] = {d.nx, d.ny, d.nz};
    for (int a = 0; a < 3; ++a)
      if (d.periodic[a] && ndc[a] < 2)
        return fail(DGMF_UNSUPPORTED, "mesh_create: store_qp_metric needs >= 2 cells in periodic direction %d", a);
  }
  const int64_t n = d.degree + 1;
  const int64_t ncells = static_cast<int64_t>(d.nx) * d.ny * d.nz;
  if (ncells > (int64_t(1) << 40) / (n * n * n)) return fail(DGMF_INVALID, "mesh_create: mesh too large");
  auto* m = new (std::nothrow) dgmf_mesh_;
  if (!m) return fail(DGMF_OOM, "mesh_create: host allocation failed");
  m->desc = d;
  m->shear = sh;
  m->desc.store_qp_metric = d.store_qp_metric ? 1 : 0;
  for (int a = 0; a < 3; ++a) m->desc.periodic[a] = d.periodic[a] ? 1 : 0;
  for (int f = 0; f < 6; ++f) m->desc.neumann[f] = (neumann_mask(m->desc) >> f) & 1;
  m->ncells = ncells;
  m->ndofs = ncells * n * n * n;
  if (hipGetDevice(&m->device) != hipSuccess) {
    delete m;
    return fail(DGMF_HIP_ERROR, "mesh_create: no HIP device");
  }
  const int nd[3] = {d.nx, d.ny, d.nz};
  const double len[3] = {d.lx, d.ly, d.lz};
  const double org[3] = {0.0, d.y0, 0.0};
  for (int a = 0; a < 3; ++a) {
    auto& v = m->verts[a];
    v.resize(nd[a] + 1);
    for (int c = 0; c <= nd[a]; ++c) {
      const double t = static_cast<double>(c) / nd[a];
      if (a == 1 && d.y_tanh_gamma > 0)
        v[c] = org[a] + 0.5 * len[a] * (1.0 + std::tanh(d.y_tanh_gamma * (2.0 * t - 1.0)) / std::tanh(d.y_tanh_gamma));
      else
        v[c] = org[a] + len[a] * t;
    }
    v[0] = org[a];
    v[nd[a]] = org[a] + len[a];
  }
  make_tables(d.degree, d.degree + 1, m->tab);
  dgmf_status st = upload_geometry<double>(m, m->geo64, m->g64);
  if (st == DGMF_OK) st = upload_geometry<float>(m, m->geo32, m->g32);
  if (st == DGMF_OK) st = upload_tables<double>(m->tab, m->tab64);
  if (st == DGMF_OK) {
    std::vector<double> mi;
    if (!inverse_mass_1d(m->tab, mi)) st = fail(DGMF_INVALID, "mesh_create: singular interpolation matrix");
    std::vector<float> mi32(mi.begin(), mi.end());
    if (st == DGMF_OK) st = m->minv64.upload(mi.data(), mi.size() * sizeof(double));
    if (st == DGMF_OK) st = m->minv32.upload(mi32.data(), mi32.size() * sizeof(float));
    if (st == DGMF_OK && d.curve_amp != 0.0) {
      // S, S^T, S^{-T}, S^{-1} for the point-weight mass of curved cells
      std::vector<long double> si;
      if (!invert(static_cast<int>(n), m->tab.S.data(), si))
        st = fail(DGMF_INVALID, "mesh_create: singular interpolation matrix");
      std::vector<double> pm(4 * n * n);
      for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
          pm[i * n + j] = m->tab.S[i * n + j];
          pm[n * n + i * n + j] = m->tab.S[j * n + i];
          if (st == DGMF_OK) {
            pm[2 * n * n + i * n + j] = static_cast<double>(si[j * n + i]);
            pm[3 * n * n + i * n + j] = static_cast<double>(si[i * n + j]);
          }
        }
      std::vector<float> pm32(pm.begin(), pm.end());
      if (st == DGMF_OK) st = m->pmt64.upload(pm.data(), pm.size() * sizeof(double));
      if (st == DGMF_OK) st = m->pmt32.upload(pm32.data(), pm32.size() * sizeof(float));
    }
    // V3c tables: Mh, Ch, Mh^{-1}, S, D, w, gw
    const Tables1D& t = m->tab;
    const V3Tab L{static_cast<int>(n)};
    std::vector<double> v3(L.size(), 0.0);
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        long double c = 0;
        for (int q = 0; q < t.nq; ++q)
          c += static_cast<long double>(t.wq[q]) * t.D[q * n + i] * t.S[q * n + j];
        v3[L.Mh() + i * n + j] = t.Mhat[i * n + j];
        v3[L.Ch() + i * n + j] = static_cast<double>(c);
        if (st == DGMF_OK) v3[L.Mi() + i * n + j] = mi[i * n + j];
        v3[L.S() + i * n + j] = t.S[i * n + j];
        v3[L.D() + i * n + j] = t.D[i * n + j];
      }
    for (int i = 0; i < n; ++i) {
      v3[L.w() + i] = t.wq[i];
      v3[L.gw() + i] = t.gll_w[i];
      v3[L.g0() + i] = t.g0[i];
      v3[L.g1() + i] = t.g1[i];
      std::vector<double> der(n);
      lagrange_eval(t.nodes, t.nodes[i], nullptr, der.data());
      for (int j = 0; j < n; ++j) {
        v3[L.Kh() + i * n + j] = t.Khat[i * n + j];
        v3[L.Dn() + i * n + j] = der[j];
      }
    }
    std::vector<float> mh32(t.Mhat.begin(), t.Mhat.end());
    if (st == DGMF_OK) st = m->v3tab.upload(v3.data(), v3.size() * sizeof(double));
    if (st == DGMF_OK) st = m->mh32.upload(mh32.data(), mh32.size() * sizeof(float));
  }
  if (st == DGMF_OK && m->desc.store_qp_metric) {
    DeviceGuard dg(m->device);
    st = setup_metric(m);
  }
  if (st != DGMF_OK) {
    delete m;
    return st;
  }
  m->g64.tab = static_cast<const double*>(m->tab64.p);
  *out = m;
  return DGMF_OK;
}

dgmf_status dgmf_mesh_info(dgmf_mesh mesh, int64_t* n_cells, int64_t* n_dofs) {
  if (!mesh) return fail(DGMF_INVALID, "mesh_info: null mesh");
  if (n_cells) *n_cells = mesh->ncells;
  if (n_dofs) *n_dofs = mesh->ndofs;
  return DGMF_OK;
}

dgmf_status dgmf_mesh_destroy(dgmf_mesh mesh) {
  if (!mesh) return DGMF_OK;
  if (mesh->nops > 0) return fail(DGMF_INVALID, "mesh_destroy: %d operator(s) still use this mesh", mesh->nops);
  DeviceGuard g(mesh->device);
  delete mesh;
  return DGMF_OK;
}

static dgmf_status flat_check(dgmf_mesh mesh, const char* who) {
  if (mesh->desc.curve_amp != 0.0) return fail(DGMF_UNSUPPORTED, "%s: curved cells are not supported", who);
  return DGMF_OK;
}

static void curved_box(dgmf_mesh mesh, double lo[3], double len[3]) {
  lo[0] = 0.0;
  lo[1] = mesh->desc.y0;
  lo[2] = 0.0;
  len[0] = mesh->desc.lx;
  len[1] = mesh->desc.ly;
  len[2] = mesh->desc.lz;
}

dgmf_status dgmf_mesh_node_coords(dgmf_mesh mesh, double* xyz, hipStream_t stream) {
  if (!mesh || !xyz) return fail(DGMF_INVALID, "mesh_node_coords: null argument");
  if (!aligned(xyz, 8)) return fail(DGMF_INVALID, "mesh_node_coords: misaligned output");
  DeviceGuard dg(mesh->device);
  if (mesh->desc.curve_amp != 0.0) {
    double lo[3], len[3];
    curved_box(mesh, lo, len);
    return launch_curved_coords(mesh->tab.n, mesh->tab.n, false, mesh->g64, lo, len, mesh->desc.curve_amp, xyz,
                                mesh->ncells, stream);
  }
  return launch_node_coords(mesh->tab.n, mesh->g64, mesh->shear, xyz, mesh->ncells, stream);
}

// curved cells: the point-weight form with w_q det J_q from the stored cell metric
static dgmf_status point_mass(dgmf_mesh mesh, dgmf_dtype dtype, int n_fields, const void* src, void* dst, bool inv,
                              hipStream_t stream) {
  const int n = mesh->tab.n;
  if (dtype == DGMF_F64)
    return launch_point_mass<double>(n, static_cast<const double*>(mesh->pmt64.p), mesh->mg64.cm,
                                     static_cast<const double*>(src), static_cast<double*>(dst), mesh->ncells,
                                     n_fields, inv, stream);
  return launch_point_mass<float>(n, static_cast<const float*>(mesh->pmt32.p), mesh->mg32.cm,
                                  static_cast<const float*>(src), static_cast<float*>(dst), mesh->ncells, n_fields,
                                  inv, stream);
}

dgmf_status dgmf_inverse_mass_apply(dgmf_mesh mesh, dgmf_dtype dtype, int n_fields, const void* src, void* dst,
                                    hipStream_t stream) {
  if (!mesh || !src || !dst) return fail(DGMF_INVALID, "inverse_mass_apply: null argument");
  const size_t es = dtype == DGMF_F64 ? 8 : (dtype == DGMF_F32 ? 4 : 0);
  if (!es) return fail(DGMF_INVALID, "inverse_mass_apply: unknown dtype %d", static_cast<int>(dtype));
  if (n_fields < 1 || n_fields > 64) return fail(DGMF_INVALID, "inverse_mass_apply: n_fields must be in 1..64");
  if (!aligned(src, es) || !aligned(dst, es)) return fail(DGMF_INVALID, "inverse_mass_apply: misaligned vector");
  if (src != dst && overlap(src, dst, es * mesh->ndofs * n_fields))
    return fail(DGMF_INVALID, "inverse_mass_apply: src and dst overlap without being the same array");
  DeviceGuard dg(mesh->device);
  const double js = 1.0 / std::fabs(mesh->shear.det);
  const int n = mesh->tab.n;
  if (mesh->desc.curve_amp != 0.0) return point_mass(mesh, dtype, n_fields, src, dst, true, stream);
  if (dtype == DGMF_F64)
    return launch_block_mass<double>(n, mesh->g64, js, static_cast<const double*>(mesh->minv64.p),
                                     static_cast<const double*>(src), static_cast<double*>(dst), mesh->ncells,
                                     n_fields, true, stream);
  return launch_block_mass<float>(n, mesh->g32, static_cast<float>(js), static_cast<const float*>(mesh->minv32.p),
                                  static_cast<const float*>(src), static_cast<float*>(dst), mesh->ncells, n_fields,
                                  true, stream);
}

dgmf_status dgmf_mass_apply(dgmf_mesh mesh, dgmf_dtype dtype, int n_fields, const void* src, void* dst,
                            hipStream_t stream) {
  if (!mesh || !src || !dst) return fail(DGMF_INVALID, "mass_apply: null argument");
  const size_t es = dtype == DGMF_F64 ? 8 : (dtype == DGMF_F32 ? 4 : 0);
  if (!es) return fail(DGMF_INVALID, "mass_apply: unknown dtype %d", static_cast<int>(dtype));
  if (n_fields < 1 || n_fields > 64) return fail(DGMF_INVALID, "mass_apply: n_fields must be in 1..64");
  if (!aligned(src, es) || !aligned(dst, es)) return fail(DGMF_INVALID, "mass_apply: misaligned vector");
  if (src != dst && overlap(src, dst, es * mesh->ndofs * n_fields))
    return fail(DGMF_INVALID, "mass_apply: src and dst overlap without being the same array");
  DeviceGuard dg(mesh->device);
  const double js = std::fabs(mesh->shear.det);
  const int n = mesh->tab.n;
  if (mesh->desc.curve_amp != 0.0) return point_mass(mesh, dtype, n_fields, src, dst, false, stream);
  if (dtype == DGMF_F64)
    return launch_block_mass<double>(n, mesh->g64, js, static_cast<const double*>(mesh->v3tab.p),
                                     static_cast<const double*>(src), static_cast<double*>(dst), mesh->ncells,
                                     n_fields, false, stream);
  return launch_block_mass<float>(n, mesh->g32, static_cast<float>(js), static_cast<const float*>(mesh->mh32.p),
                                  static_cast<const float*>(src), static_cast<float*>(dst), mesh->ncells, n_fields,
                                  false, stream);
}

// Neumann sides need no check here: the ND average is the own trace on both
// boundary parts (A, B), and the viscous coupling kernel skips Neumann faces.
// Rows the curved-cell metric fill needs after a table's S, D and weights: the
// GLL nodes, l(0) and l(1) (unit vectors: the end points are nodes), l'(0)
// and l'(1); off receives their offsets {nodes, l(0), l'(0)}.
static void append_curved_rows(const dgmf::Tables1D& t, std::vector<double>& h, int off[3]) {
  const int n = t.n;
  off[0] = static_cast<int>(h.size());
  h.insert(h.end(), t.nodes.begin(), t.nodes.end());
  off[1] = static_cast<int>(h.size());
  h.resize(h.size() + 2 * n, 0.0);
  h[off[1]] = 1.0;
  h[off[1] + 2 * n - 1] = 1.0;
  off[2] = static_cast<int>(h.size());
  h.insert(h.end(), t.g0.begin(), t.g0.end());
  h.insert(h.end(), t.g1.begin(), t.g1.end());
}

static dgmf_status v3_check(dgmf_mesh mesh, const char* who, bool curved_ok = false) {
  if (!mesh) return fail(DGMF_INVALID, "%s: null mesh", who);
  if (mesh->shear.on) return fail(DGMF_UNSUPPORTED, "%s: sheared meshes are not supported", who);
  if (!curved_ok)
    if (dgmf_status e = flat_check(mesh, who)) return e;
  return DGMF_OK;
}

// Curved cells: tables and per-point metric of the divergence and gradient at
// n_q = k+1 points, built (synchronously, on the null stream) on first use.
static dgmf_status curved_v3_geometry(dgmf_mesh mesh) {
  if (mesh->qgeo.cmet) return DGMF_OK;
  const int n = mesh->tab.n, nq = n;
  const dgmf::Tables1D& t = mesh->tab;
  std::vector<double> h;
  h.insert(h.end(), t.S.begin(), t.S.end());
  h.insert(h.end(), t.D.begin(), t.D.end());
  h.insert(h.end(), t.wq.begin(), t.wq.end());
  int rows[3];
  append_curved_rows(t, h, rows);
  // S^{-1} (S is square here) for the inverse mass of the projection
  std::vector<long double> si;
  if (!invert(n, t.S.data(), si)) return fail(DGMF_INVALID, "curved V3c: singular interpolation matrix");
  const int o_si = static_cast<int>(h.size());
  for (int i = 0; i < n * n; ++i) h.push_back(static_cast<double>(si[i]));
  dgmf_status st;
  if ((st = mesh->qtab.upload(h.data(), h.size() * sizeof(double)))) return st;
  const int64_t nq2 = static_cast<int64_t>(nq) * nq, cper = 9 * nq2 * nq, fper = 18 * nq2;
  if ((st = mesh->qmet.alloc(static_cast<size_t>(mesh->ncells * (cper + fper)) * sizeof(double)))) return st;
  double* cm = static_cast<double*>(mesh->qmet.p);
  const double* x0[3] = {mesh->g64.x0[0], mesh->g64.x0[1], mesh->g64.x0[2]};
  const double* hh[3] = {mesh->g64.h[0], mesh->g64.h[1], mesh->g64.h[2]};
  const double lo[3] = {0.0, mesh->desc.y0, 0.0};
  const double len[3] = {mesh->desc.lx, mesh->desc.ly, mesh->desc.lz};
  const int off[6] = {rows[0], 0, nq * n, 2 * nq * n, rows[1], rows[2]};
  if ((st = launch_conv_fill_curved(n, nq, x0, hh, lo, len, mesh->desc.curve_amp, mesh->g64.nx, mesh->g64.ny,
                                    mesh->ncells, static_cast<const double*>(mesh->qtab.p), off, cm,
                                    cm + mesh->ncells * cper, nullptr)))
    return st;
  DGMF_HIP_TRY(hipStreamSynchronize(nullptr));
  ConvGeom& g = mesh->qgeo;
  g.nx = mesh->g64.nx;
  g.ny = mesh->g64.ny;
  g.nz = mesh->g64.nz;
  g.neu = neumann_mask(mesh->desc);
  for (int d = 0; d < 3; ++d) {
    g.per[d] = mesh->g64.per[d];
    g.h[d] = mesh->g64.h[d];
    g.hinv[d] = mesh->g64.hinv[d];
  }
  g.tab = static_cast<const double*>(mesh->qtab.p);
  g.S = 0;
  g.D = nq * n;
  g.w = 2 * nq * n;
  g.Mi = o_si;   // S^{-1}
  g.fmet = cm + mesh->ncells * cper;
  g.cmet = cm;
  return DGMF_OK;
}

// Curved cells: 1D tables of the viscous coupling (S, D, w at the k+1 Gauss
// points, then the GLL nodes, l(0) l(1) and l'(0) l'(1)), uploaded on first use.
static dgmf_status curved_eps_tables(dgmf_mesh mesh) {
  if (mesh->egeo.tab) return DGMF_OK;
  const int n = mesh->tab.n, nq = n;
  const dgmf::Tables1D& t = mesh->tab;
  std::vector<double> h;
  h.insert(h.end(), t.S.begin(), t.S.end());
  h.insert(h.end(), t.D.begin(), t.D.end());
  h.insert(h.end(), t.wq.begin(), t.wq.end());
  int rows[3];
  append_curved_rows(t, h, rows);
  dgmf_status st;
  if ((st = mesh->etab.upload(h.data(), h.size() * sizeof(double)))) return st;
  ConvGeom& g = mesh->egeo;
  g.nx = mesh->g64.nx;
  g.ny = mesh->g64.ny;
  g.nz = mesh->g64.nz;
  g.neu = neumann_mask(mesh->desc);
  for (int d = 0; d < 3; ++d) {
    g.per[d] = mesh->g64.per[d];
    g.h[d] = mesh->g64.h[d];
    g.hinv[d] = mesh->g64.hinv[d];
  }
  g.S = 0;
  g.D = nq * n;
  g.w = 2 * nq * n;
  g.Mi = 0;
  g.cmet = g.fmet = nullptr;
  for (int k = 0; k < 3; ++k) mesh->eoff[k] = rows[k];
  g.tab = static_cast<const double*>(mesh->etab.p);
  return DGMF_OK;
}

// out = H_eps u on curved cells: the stored-metric scalar apply per component, then the coupling
static dgmf_status viscous_apply_curved(dgmf_op op, const double* u, double* out, hipStream_t stream) {
  dgmf_mesh mesh = op->mesh;
  dgmf_status e = curved_eps_tables(mesh);
  if (e) return e;
  const int64_t N = mesh->ndofs;
  for (int a = 0; a < 3; ++a)
    if ((e = sipg_apply<double>(op, u + a * N, out + a * N, nullptr, nullptr, stream))) return e;
  const double* x0[3] = {mesh->g64.x0[0], mesh->g64.x0[1], mesh->g64.x0[2]};
  const double* hh[3] = {mesh->g64.h[0], mesh->g64.h[1], mesh->g64.h[2]};
  const double lo[3] = {0.0, mesh->desc.y0, 0.0};
  const double len[3] = {mesh->desc.lx, mesh->desc.ly, mesh->desc.lz};
  return launch_eps_curved(mesh->tab.n, mesh->egeo, x0, hh, lo, len, mesh->desc.curve_amp, mesh->eoff[0],
                           mesh->eoff[1], mesh->eoff[2], u, out, op->sipg.diff_coeff, mesh->ncells, stream);
}

}  // extern "C"

namespace dgmf {
dgmf_status viscous_apply_any(dgmf_op op, const double* u, double* out, hipStream_t stream) {
  if (op->mesh->desc.curve_amp != 0.0) return viscous_apply_curved(op, u, out, stream);
  const int64_t N = op->mesh->ndofs;
  for (int a = 0; a < 3; ++a)
    if (dgmf_status e = sipg_apply<double>(op, u + a * N, out + a * N, nullptr, nullptr, stream)) return e;
  return launch_eps_coupling(op->mesh->tab.n, op->mesh->g64, static_cast<const double*>(op->mesh->v3tab.p), u, out,
                             op->sipg.diff_coeff, op->mesh->ncells, stream);
}
}  // namespace dgmf

extern "C" {

dgmf_status dgmf_viscous_apply(dgmf_op op, const double* u, double* out, hipStream_t stream) {
  if (!op || op->kind != 1) return fail(DGMF_INVALID, "viscous_apply: not an SIPG operator");
  dgmf_status e = v3_check(op->mesh, "viscous_apply", true);
  if (e) return e;
  if (!u || !out || !aligned(u, 8) || !aligned(out, 8))
    return fail(DGMF_INVALID, "viscous_apply: null or misaligned vector");
  const int64_t N = op->mesh->ndofs;
  if (overlap(u, out, 24 * N)) return fail(DGMF_INVALID, "viscous_apply: u and out overlap");
  DeviceGuard dg(op->mesh->device);
  return viscous_apply_any(op, u, out, stream);
}

dgmf_status dgmf_divergence_apply(dgmf_mesh mesh, const double* u, double* out, hipStream_t stream) {
  dgmf_status e = v3_check(mesh, "divergence_apply", true);
  if (e) return e;
  if (!u || !out || !aligned(u, 8) || !aligned(out, 8))
    return fail(DGMF_INVALID, "divergence_apply: null or misaligned vector");
  if (overlap2(u, 24 * mesh->ndofs, out, 8 * mesh->ndofs))
    return fail(DGMF_INVALID, "divergence_apply: u and out overlap");
  DeviceGuard dg(mesh->device);
  if (mesh->desc.curve_amp != 0.0) {
    if ((e = curved_v3_geometry(mesh))) return e;
    return launch_curv_v3(mesh->tab.n, false, mesh->qgeo, u, out, mesh->ncells, stream);
  }
  return launch_v3_divergence(mesh->tab.n, mesh->g64, static_cast<const double*>(mesh->v3tab.p), u, out,
                              mesh->ncells, stream);
}

dgmf_status dgmf_gradient_apply(dgmf_mesh mesh, const double* p, double* out, hipStream_t stream) {
  dgmf_status e = v3_check(mesh, "gradient_apply", true);
  if (e) return e;
  if (!p || !out || !aligned(p, 8) || !aligned(out, 8))
    return fail(DGMF_INVALID, "gradient_apply: null or misaligned vector");
  if (overlap2(p, 8 * mesh->ndofs, out, 24 * mesh->ndofs))
    return fail(DGMF_INVALID, "gradient_apply: p and out overlap");
  DeviceGuard dg(mesh->device);
  if (mesh->desc.curve_amp != 0.0) {
    if ((e = curved_v3_geometry(mesh))) return e;
    return launch_curv_v3(mesh->tab.n, true, mesh->qgeo, p, out, mesh->ncells, stream);
  }
  return launch_v3_gradient(mesh->tab.n, mesh->g64, static_cast<const double*>(mesh->v3tab.p), p, out, mesh->ncells,
                            stream);
}

dgmf_status dgmf_divdiv_penalty(dgmf_mesh mesh, const double* u, double zeta, double dt, double* tau,
                                hipStream_t stream) {
  dgmf_status e = v3_check(mesh, "divdiv_penalty", true);
  if (e) return e;
  if (!u || !tau || !aligned(u, 8) || !aligned(tau, 8))
    return fail(DGMF_INVALID, "divdiv_penalty: null or misaligned vector");
  if (!std::isfinite(zeta) || !std::isfinite(dt) || zeta < 0 || dt < 0)
    return fail(DGMF_INVALID, "divdiv_penalty: zeta and dt must be finite and >= 0");
  if (overlap2(u, 24 * mesh->ndofs, tau, 8 * mesh->ncells))
    return fail(DGMF_INVALID, "divdiv_penalty: u and tau overlap");
  DeviceGuard dg(mesh->device);
  if (mesh->desc.curve_amp != 0.0) {
    if ((e = curved_v3_geometry(mesh))) return e;
    return launch_curv_cell(mesh->tab.n, false, mesh->qgeo, mesh->mg64.cm, u, zeta, dt, tau, nullptr, nullptr, nullptr,
                            0.0, 0, nullptr, mesh->ncells, stream);
  }
  return launch_v3_tau(mesh->tab.n, mesh->g64, static_cast<const double*>(mesh->v3tab.p), u, zeta, dt, tau,
                       mesh->ncells, stream);
}

dgmf_status dgmf_projection_solve(dgmf_mesh mesh, const double* tau, const double* rhs, double* x, double rtol,
                                  int max_iter, int* iterations, hipStream_t stream) {
  dgmf_status e = v3_check(mesh, "projection_solve", true);
  if (e) return e;
  if (!v3_projection_supported(mesh->tab.n))
    return fail(DGMF_UNSUPPORTED, "projection_solve: degree %d not built (k <= 6)", mesh->tab.n - 1);
  if (!tau || !rhs || !x || !aligned(tau, 8) || !aligned(rhs, 8) || !aligned(x, 8) ||
      (iterations && !aligned(iterations, 4)))
    return fail(DGMF_INVALID, "projection_solve: null or misaligned argument");
  if (!(rtol >= 0) || !std::isfinite(rtol) || max_iter < 0)
    return fail(DGMF_INVALID, "projection_solve: rtol must be finite and >= 0, max_iter >= 0");
  const size_t vb = 24 * mesh->ndofs, tb = 8 * mesh->ncells, ib = 4 * mesh->ncells;
  if (overlap2(rhs, vb, x, vb) || overlap2(tau, tb, x, vb) || (iterations && overlap2(iterations, ib, x, vb)))
    return fail(DGMF_INVALID, "projection_solve: x overlaps another argument");
  DeviceGuard dg(mesh->device);
  if (mesh->desc.curve_amp != 0.0) {
    if ((e = curved_v3_geometry(mesh))) return e;
    return launch_curv_cell(mesh->tab.n, true, mesh->qgeo, mesh->mg64.cm, nullptr, 0.0, 0.0, nullptr, tau, rhs, x,
                            rtol, max_iter, iterations, mesh->ncells, stream);
  }
  return launch_v3_projection(mesh->tab.n, mesh->g64, static_cast<const double*>(mesh->v3tab.p), tau, rhs, x, rtol,
                              max_iter, iterations, mesh->ncells, stream);
}

dgmf_status dgmf_sipg_create(dgmf_mesh mesh, const dgmf_sipg_desc* desc, dgmf_op* out) {
  if (!mesh || !desc || !out) return fail(DGMF_INVALID, "sipg_create: null argument");
  const int n = mesh->desc.degree + 1;
  if (desc->n_q != 0 && desc->n_q != n)
    return fail(DGMF_UNSUPPORTED, "sipg_create: n_q must be 0 or k+1 (got %d)", desc->n_q);
  if (mesh->ndofs >= (int64_t(1) << 31))
    return fail(DGMF_UNSUPPORTED, "sipg_create: %lld DoF per field exceed the 32-bit indexing of the kernels",
                static_cast<long long>(mesh->ndofs));
  if (!std::isfinite(desc->mass_coeff) || !std::isfinite(desc->diff_coeff) || !std::isfinite(desc->penalty_scale) ||
      desc->mass_coeff < 0 || desc->diff_coeff < 0 || !(desc->penalty_scale > 0))
    return fail(DGMF_INVALID, "sipg_create: coefficients must be finite, mass/diff >= 0, penalty > 0");
  DeviceGuard dg(mesh->device);
  auto* op = new (std::nothrow) dgmf_op_;
  if (!op) return fail(DGMF_OOM, "sipg_create: host allocation failed");
  op->kind = 1;
  op->mesh = mesh;
  op->sipg = *desc;
  op->nq = n;
  make_tables(mesh->desc.degree, n, op->tab);
  // x-line operator with the mass term folded in when the x spacing is uniform:
  // nu hy hz/hx Khat + mu hx hy hz Mhat = (nu hy hz/hx) (Khat + (mu hx^2/nu) Mhat)
  const auto& vx = mesh->verts[0];
  bool uniform_x = true;
  const double hx0 = vx[1] - vx[0];
  for (size_t c = 1; c + 1 < vx.size(); ++c)
    if (std::fabs((vx[c + 1] - vx[c]) - hx0) > 1e-14 * hx0) uniform_x = false;
  std::vector<double> xhat(n * n);
  for (int i = 0; i < n * n; ++i)
    xhat[i] = desc->diff_coeff > 0 ? op->tab.Khat[i] + desc->mass_coeff * hx0 * hx0 / desc->diff_coeff * op->tab.Mhat[i]
                                   : op->tab.Mhat[i];
  dgmf_status st = upload_tables<double>(op->tab, op->tab64, &xhat);
  if (st == DGMF_OK) st = upload_tables<float>(op->tab, op->tab32, &xhat);
  op->g64 = mesh->g64;
  op->g32 = mesh->g32;
  const int allper = mesh->desc.periodic[0] && mesh->desc.periodic[1] && mesh->desc.periodic[2];
  op->g64.xcomb = op->g32.xcomb = uniform_x ? 1 : 0;
  op->g64.allper = op->g32.allper = allper;
  if (st != DGMF_OK) {
    delete op;
    return st;
  }
  const double pen = desc->penalty_scale * n * n;
  // uniform spacing in every direction and every direction periodic: pre-scaled line operators
  op->g64.utab = nullptr;
  op->g32.utab = nullptr;
  if (allper && !mesh->desc.store_qp_metric) {
    bool uni = true;
    double hu[3];
    for (int a = 0; a < 3 && uni; ++a) {
      const auto& v = mesh->verts[a];
      hu[a] = v[1] - v[0];
      for (size_t c = 1; c + 1 < v.size(); ++c)
        if (std::fabs((v[c + 1] - v[c]) - hu[a]) > 1e-14 * hu[a]) uni = false;
    }
    if (uni) {
      st = upload_uniform_tables<double>(op->tab, hu, desc->mass_coeff, desc->diff_coeff, pen, op->utab64);
      if (st == DGMF_OK)
        st = upload_uniform_tables<float>(op->tab, hu, desc->mass_coeff, desc->diff_coeff, pen, op->utab32);
      if (st != DGMF_OK) {
        delete op;
        return st;
      }
      op->g64.utab = static_cast<const double*>(op->utab64.p);
      op->g32.utab = static_cast<const float*>(op->utab32.p);
    }
  }
  op->g64.pen = pen;
  op->g64.mu = desc->mass_coeff;
  op->g64.nu = desc->diff_coeff;
  op->g64.tab = static_cast<const double*>(op->tab64.p);
  op->g32.pen = static_cast<float>(pen);
  op->g32.mu = static_cast<float>(desc->mass_coeff);
  op->g32.nu = static_cast<float>(desc->diff_coeff);
  op->g32.tab = static_cast<const float*>(op->tab32.p);
  if (mesh->desc.store_qp_metric) {
    // stored metric: tau geometry already carries (k+1)^2
    op->metric = true;
    op->mg64 = mesh->mg64;
    op->mg32 = mesh->mg32;
    op->mg64.mu = desc->mass_coeff;
    op->mg64.nu = desc->diff_coeff;
    op->mg64.pen = desc->penalty_scale;
    op->mg32.mu = static_cast<float>(desc->mass_coeff);
    op->mg32.nu = static_cast<float>(desc->diff_coeff);
    op->mg32.pen = static_cast<float>(desc->penalty_scale);
  }
  {
    // the diagonal, computed once (Sec. 5.1: precomputed before time stepping) for the
    // Jacobi and Chebyshev preconditioners and the multigrid smoothers
    DeviceGuard dg(mesh->device);
    dgmf_status sd = op->diag64.alloc(static_cast<size_t>(mesh->ndofs) * sizeof(double));
    if (sd == DGMF_OK) sd = sipg_diag64(op, static_cast<double*>(op->diag64.p), nullptr);
    if (sd == DGMF_OK) {
      const hipError_t he = hipStreamSynchronize(nullptr);
      if (he != hipSuccess) sd = fail(DGMF_HIP_ERROR, "sipg_create: diagonal: %s", hipGetErrorString(he));
    }
    if (sd != DGMF_OK) {
      delete op;
      return sd;
    }
    // launch plans of the axis-aligned apply depend on its occupancy: query it
    // here, outside any stream capture (the multigrid V-cycle is captured)
    if (!op->metric) sipg_cart_prime(n);
  }
  mesh->nops++;
  *out = op;
  return DGMF_OK;
}

dgmf_status dgmf_operator_apply(dgmf_op op, dgmf_dtype dtype, const void* src, void* dst, hipStream_t stream) {
  if (!op || op->kind != 1) return fail(DGMF_INVALID, "operator_apply: not an SIPG operator");
  if (!src || !dst) return fail(DGMF_INVALID, "operator_apply: null vector");
  const size_t es = dtype == DGMF_F64 ? 8 : (dtype == DGMF_F32 ? 4 : 0);
  if (!es) return fail(DGMF_INVALID, "operator_apply: unknown dtype %d", static_cast<int>(dtype));
  if (!aligned(src, es) || !aligned(dst, es)) return fail(DGMF_INVALID, "operator_apply: misaligned vector");
  if (overlap(src, dst, es * op->mesh->ndofs)) return fail(DGMF_INVALID, "operator_apply: src and dst overlap");
  DeviceGuard dg(op->mesh->device);
  if (dtype == DGMF_F64)
    return sipg_apply<double>(op, static_cast<const double*>(src), static_cast<double*>(dst), nullptr, nullptr, stream);
  return sipg_apply<float>(op, static_cast<const float*>(src), static_cast<float*>(dst), nullptr, nullptr, stream);
}

dgmf_status dgmf_operator_diagonal(dgmf_op op, dgmf_dtype dtype, void* diag, hipStream_t stream) {
  if (!op || op->kind != 1) return fail(DGMF_INVALID, "operator_diagonal: not an SIPG operator");
  if (!diag) return fail(DGMF_INVALID, "operator_diagonal: null vector");
  const size_t es = dtype == DGMF_F64 ? 8 : (dtype == DGMF_F32 ? 4 : 0);
  if (!es) return fail(DGMF_INVALID, "operator_diagonal: unknown dtype %d", static_cast<int>(dtype));
  if (!aligned(diag, es)) return fail(DGMF_INVALID, "operator_diagonal: misaligned vector");
  DeviceGuard dg(op->mesh->device);
  const int n = op->mesh->desc.degree + 1;
  if (op->metric) {
    if (dtype == DGMF_F64) return launch_sipg_metric_diag<double>(n, op->mg64, static_cast<double*>(diag), stream);
    return launch_sipg_metric_diag<float>(n, op->mg64, static_cast<float*>(diag), stream);
  }
  if (dtype == DGMF_F64)
    return launch_sipg_cart_diag<double>(n, op->g64, static_cast<double*>(diag), op->mesh->ncells, stream);
  return launch_sipg_cart_diag<float>(n, op->g32, static_cast<float*>(diag), op->mesh->ncells, stream);
}

dgmf_status dgmf_quadrature_points(dgmf_op op, double* xyz, hipStream_t stream) {
  if (!op || op->kind != 1) return fail(DGMF_INVALID, "quadrature_points: not an SIPG operator");
  if (!xyz || !aligned(xyz, 8)) return fail(DGMF_INVALID, "quadrature_points: null or misaligned output");
  DeviceGuard dg(op->mesh->device);
  if (op->mesh->desc.curve_amp != 0.0) {
    double lo[3], len[3];
    curved_box(op->mesh, lo, len);
    return launch_curved_coords(op->tab.n, op->nq, true, op->g64, lo, len, op->mesh->desc.curve_amp, xyz,
                                op->mesh->ncells, stream);
  }
  return launch_qp_coords(op->tab.n, op->nq, op->g64, op->mesh->shear, xyz, op->mesh->ncells, stream);
}

dgmf_status dgmf_integrate(dgmf_op op, const double* f_qp, double* b, hipStream_t stream) {
  if (!op || op->kind != 1) return fail(DGMF_INVALID, "integrate: not an SIPG operator");
  if (!f_qp || !b || !aligned(f_qp, 8) || !aligned(b, 8))
    return fail(DGMF_INVALID, "integrate: null or misaligned vector");
  const int64_t nq3 = static_cast<int64_t>(op->nq) * op->nq * op->nq;
  if (overlap(f_qp, b, 8 * std::min<int64_t>(op->mesh->ndofs, op->mesh->ncells * nq3)))
    return fail(DGMF_INVALID, "integrate: input and output overlap");
  DeviceGuard dg(op->mesh->device);
  if (op->mesh->desc.curve_amp != 0.0)   // n_q = k+1 here (sipg_create), the rule of the stored metric
    return launch_integrate_curved(op->tab.n, op->g64.tab + TabLayout{op->tab.n, op->nq}.S(), op->mesh->mg64.cm, f_qp,
                                   b, op->mesh->ncells, stream);
  return launch_integrate(op->tab.n, op->nq, op->g64, op->mesh->shear, f_qp, b, op->mesh->ncells, stream);
}

}  // extern "C"

namespace dgmf {

template <typename T>
dgmf_status sipg_apply(dgmf_op op, const T* src, T* dst, double* partials, const int* stop, hipStream_t s) {
  const int n = op->mesh->desc.degree + 1;
  if (op->metric) {
    if constexpr (std::is_same<T, double>::value)
      return launch_sipg_metric_apply<double>(n, op->mg64, src, dst, partials, stop, s);
    else
      return launch_sipg_metric_apply<float>(n, op->mg32, src, dst, partials, stop, s);
  }
  if constexpr (std::is_same<T, double>::value)
    return launch_sipg_cart_apply<double>(n, op->g64, src, dst, op->mesh->ncells, partials, stop, s);
  else
    return launch_sipg_cart_apply<float>(n, op->g32, src, dst, op->mesh->ncells, partials, stop, s);
}
template dgmf_status sipg_apply<double>(dgmf_op, const double*, double*, double*, const int*, hipStream_t);
template dgmf_status sipg_apply<float>(dgmf_op, const float*, float*, double*, const int*, hipStream_t);

template <typename T>
dgmf_status sipg_cheb(dgmf_op op, const T* xk, T* dst, const ChebEpi<T>& epi, const int* stop, hipStream_t s) {
  const int n = op->mesh->desc.degree + 1;
  if (op->metric) {
    if constexpr (std::is_same<T, double>::value)
      return launch_sipg_metric_cheb<double>(n, op->mg64, xk, dst, epi, stop, s);
    else
      return launch_sipg_metric_cheb<float>(n, op->mg32, xk, dst, epi, stop, s);
  }
  if constexpr (std::is_same<T, double>::value)
    return launch_sipg_cart_cheb<double>(n, op->g64, xk, dst, epi, stop, s);
  else
    return launch_sipg_cart_cheb<float>(n, op->g32, xk, dst, epi, stop, s);
}
template dgmf_status sipg_cheb<double>(dgmf_op, const double*, double*, const ChebEpi<double>&, const int*,
                                       hipStream_t);
template dgmf_status sipg_cheb<float>(dgmf_op, const float*, float*, const ChebEpi<float>&, const int*, hipStream_t);

dgmf_status sipg_diag64(dgmf_op op, double* diag, hipStream_t s) {
  const int n = op->mesh->desc.degree + 1;
  if (op->metric) return launch_sipg_metric_diag<double>(n, op->mg64, diag, s);
  return launch_sipg_cart_diag<double>(n, op->g64, diag, op->mesh->ncells, s);
}

int64_t sipg_apply_blocks(dgmf_op op) {
  if (op->metric) return metric_apply_blocks(op->mesh->desc.degree + 1, op->mg64.nx, op->mg64.ny, op->mg64.nz);
  return sipg_cart_blocks(op->mesh->desc.degree + 1, op->g64);
}

}  // namespace dgmf

extern "C" {

dgmf_status dgmf_op_destroy(dgmf_op op) {
  if (!op) return DGMF_OK;
  DeviceGuard dg(op->mesh->device);
  if (op->mgh) mg_destroy(op->mgh);
  op->mesh->nops--;
  delete op;
  return DGMF_OK;
}

}  // extern "C"

extern "C" {

dgmf_status dgmf_convective_create(dgmf_mesh mesh, const dgmf_conv_desc* desc, dgmf_op* out) {
  if (!mesh || !desc || !out) return fail(DGMF_INVALID, "convective_create: null argument");
  const int k = mesh->desc.degree, n = k + 1;
  const int nq = desc->n_q > 0 ? desc->n_q : (3 * (k + 1)) / 2;
  if (desc->n_q < 0) return fail(DGMF_INVALID, "convective_create: n_q must be >= 0");
  if (mesh->shear.on) return fail(DGMF_UNSUPPORTED, "convective_create: sheared meshes are not supported");
  if (!conv_supported(n, nq))
    return fail(DGMF_UNSUPPORTED, "convective_create: degree %d with %d points per direction not built", k, nq);
  DeviceGuard dg(mesh->device);
  auto* op = new (std::nothrow) dgmf_op_;
  if (!op) return fail(DGMF_OOM, "convective_create: host allocation failed");
  op->kind = 2;
  op->mesh = mesh;
  op->nq = nq;
  make_tables(k, nq, op->tab);
  std::vector<double> h;
  h.insert(h.end(), op->tab.S.begin(), op->tab.S.end());
  h.insert(h.end(), op->tab.D.begin(), op->tab.D.end());
  h.insert(h.end(), op->tab.wq.begin(), op->tab.wq.end());
  std::vector<double> mi;
  if (!inverse_mass_1d(mesh->tab, mi)) {
    delete op;
    return fail(DGMF_INVALID, "convective_create: singular interpolation matrix");
  }
  h.insert(h.end(), mi.begin(), mi.end());
  int rows[3];   // for the curved-cell metric fill
  append_curved_rows(op->tab, h, rows);
  dgmf_status st = op->ctab.upload(h.data(), h.size() * sizeof(double));
  if (st != DGMF_OK) {
    delete op;
    return st;
  }
  ConvGeom& g = op->cgeo;
  g.cmet = nullptr;
  g.fmet = nullptr;
  if (mesh->desc.curve_amp != 0.0) {
    // per point: 9 cell values, 6 faces x 3 normal components
    const int64_t nq2 = static_cast<int64_t>(nq) * nq, cper = 9 * nq2 * nq, fper = 18 * nq2;
    if ((st = op->cmet.alloc(static_cast<size_t>(mesh->ncells * (cper + fper)) * sizeof(double)))) {
      delete op;
      return st;
    }
    double* cm = static_cast<double*>(op->cmet.p);
    const double* x0[3] = {mesh->g64.x0[0], mesh->g64.x0[1], mesh->g64.x0[2]};
    const double* hh[3] = {mesh->g64.h[0], mesh->g64.h[1], mesh->g64.h[2]};
    const double lo[3] = {0.0, mesh->desc.y0, 0.0};
    const double len[3] = {mesh->desc.lx, mesh->desc.ly, mesh->desc.lz};
    const int off[6] = {rows[0], 0, nq * n, 2 * nq * n, rows[1], rows[2]};
    st = launch_conv_fill_curved(n, nq, x0, hh, lo, len, mesh->desc.curve_amp, mesh->g64.nx, mesh->g64.ny,
                                 mesh->ncells, static_cast<const double*>(op->ctab.p), off, cm,
                                 cm + mesh->ncells * cper, nullptr);
    if (st == DGMF_OK && hipStreamSynchronize(nullptr) != hipSuccess)
      st = fail(DGMF_HIP_ERROR, "convective_create: curved metric fill failed");
    if (st != DGMF_OK) {
      delete op;
      return st;
    }
    g.cmet = cm;
    g.fmet = cm + mesh->ncells * cper;
  }
  g.neu = neumann_mask(mesh->desc);
  g.nx = mesh->g64.nx;
  g.ny = mesh->g64.ny;
  g.nz = mesh->g64.nz;
  for (int d = 0; d < 3; ++d) {
    g.per[d] = mesh->g64.per[d];
    g.h[d] = mesh->g64.h[d];
    g.hinv[d] = mesh->g64.hinv[d];
  }
  g.tab = static_cast<const double*>(op->ctab.p);
  g.S = 0;
  g.D = nq * n;
  g.w = 2 * nq * n;
  g.Mi = 2 * nq * n + nq;
  mesh->nops++;
  *out = op;
  return DGMF_OK;
}

dgmf_status dgmf_convective_apply(dgmf_op op, const double* u, double* out, hipStream_t stream) {
  if (!op || op->kind != 2) return fail(DGMF_INVALID, "convective_apply: not a convective operator");
  if (!u || !out || !aligned(u, 8) || !aligned(out, 8))
    return fail(DGMF_INVALID, "convective_apply: null or misaligned vector");
  if (overlap(u, out, 24 * op->mesh->ndofs)) return fail(DGMF_INVALID, "convective_apply: u and out overlap");
  DeviceGuard dg(op->mesh->device);
  return launch_conv_fwd(op->tab.n, op->nq, op->cgeo, u, out, op->mesh->ncells, false, 0.0, stream);
}

dgmf_status dgmf_convective_step(dgmf_op op, double dt, const double* u, double* out, hipStream_t stream) {
  if (!op || op->kind != 2) return fail(DGMF_INVALID, "convective_step: not a convective operator");
  if (!std::isfinite(dt)) return fail(DGMF_INVALID, "convective_step: dt must be finite");
  if (!u || !out || !aligned(u, 8) || !aligned(out, 8))
    return fail(DGMF_INVALID, "convective_step: null or misaligned vector");
  if (overlap(u, out, 24 * op->mesh->ndofs)) return fail(DGMF_INVALID, "convective_step: u and out overlap");
  if (op->cgeo.cmet) return fail(DGMF_UNSUPPORTED, "convective_step: curved cells are not supported");
  DeviceGuard dg(op->mesh->device);
  return launch_conv_fwd(op->tab.n, op->nq, op->cgeo, u, out, op->mesh->ncells, true, dt, stream);
}

dgmf_status dgmf_convective_vjp(dgmf_op op, const double* u, const double* w, double* grad, hipStream_t stream) {
  if (!op || op->kind != 2) return fail(DGMF_INVALID, "convective_vjp: not a convective operator");
  if (!u || !w || !grad || !aligned(u, 8) || !aligned(w, 8) || !aligned(grad, 8))
    return fail(DGMF_INVALID, "convective_vjp: null or misaligned vector");
  const size_t bytes = 24 * op->mesh->ndofs;
  if (overlap(u, grad, bytes) || overlap(w, grad, bytes))
    return fail(DGMF_INVALID, "convective_vjp: grad overlaps u or w");
  DeviceGuard dg(op->mesh->device);
  return launch_conv_vjp(op->tab.n, op->nq, op->cgeo, u, w, grad, op->mesh->ncells, stream);
}

}  // extern "C"
