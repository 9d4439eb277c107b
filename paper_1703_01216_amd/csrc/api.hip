// C-ABI of the solver (declared in include/fr3d.h): context, workspaces,
// kernel spectrum, data transform, alpha evaluations and search, recovery,
// source potential, forward operator and noise.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fr3d.h"
#include "control.hpp"
#include "passes.hpp"

using namespace fr3d;

// ============================================================ small kernels
namespace {

__global__ void k_ctrl_init(Ctrl* c, Ctrl v) { *c = v; }

// zeta = xi V0 is not formed here; recovery: xi = zeta / V0 and
// c = (1/c0^2 - xi)^(-1/2) with the argument clamped at 1e-6/c0^2.
template <typename T>
__global__ void k_recover(const T* __restrict__ zeta, const T* __restrict__ V0, double inv_c02, double floor_,
                          T* __restrict__ c, long long n, double* part) {
  __shared__ double red[NT / 64];
  double cl = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const double xi = (double)zeta[i] / (double)V0[i];
    double arg = inv_c02 - xi;
    if (arg < floor_) { arg = floor_; cl += 1.0; }
    c[i] = (T)(1.0 / sqrt(arg));
  }
  cl = block_sum<NT>(cl, red);
  if (threadIdx.x == 0) part[blockIdx.x] = cl;
}

// out[j] = sum over k < nblk of part[k*stride + j] for j < nout (one workgroup).
__global__ void k_sum_parts(const double* __restrict__ part, int nblk, int stride, int nout, double* out) {
  __shared__ double red[NT / 64];
  for (int j = 0; j < nout; ++j) {
    double s = 0.0;
    for (int k = threadIdx.x; k < nblk; k += NT) s += part[(size_t)k * stride + j];
    s = block_sum<NT>(s, red);
    if (threadIdx.x == 0) out[j] = s;
  }
}

// V0(x) = -(A0/4 pi) sum_l 1/|x - x_l| at R's cell centres (Sec. 6 point sources).
struct Sources { double x[10], y[10], z[10]; };

template <typename T>
__global__ void k_v0(T* __restrict__ V0, int nx, int ny, int nz, double h, double A0, Sources s) {
  const long long n = (long long)nx * ny * nz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((long long)nx * ny));
    const double px = (ix + 0.5) * h, py = (iy + 0.5) * h, pz = (iz + 0.5) * h;
    double acc = 0.0;
    for (int l = 0; l < 10; ++l) {
      const double dx = px - s.x[l], dy = py - s.y[l], dz = pz - s.z[l];
      acc += 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    }
    V0[i] = (T)(-(A0 / (4.0 * M_PI)) * acc);
  }
}

// Sum of squares of two arrays in FP64, per-block partials (summed in a fixed
// order by k_sum_parts): part[2 blk] = ||a||^2 part, part[2 blk + 1] = ||b||^2 part.
template <typename T>
__global__ void k_norms2(const T* __restrict__ a, const T* __restrict__ b, long long n, double* part) {
  __shared__ double red[NT / 64];
  double sa = 0.0, sb = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const double va = a[i], vb = b[i];
    sa += va * va;
    sb += vb * vb;
  }
  sa = block_sum<NT>(sa, red);
  sb = block_sum<NT>(sb, red);
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sa;
    part[2 * blockIdx.x + 1] = sb;
  }
}

// F += e * (delta_rel ||F|| / ||e||); the factor comes from nrm = (||F||^2, ||e||^2).
template <typename T>
__global__ void k_add_noise(T* __restrict__ F, const T* __restrict__ e, long long n, double delta_rel,
                            const double* nrm) {
  const double f = delta_rel * sqrt(nrm[0]) / sqrt(nrm[1]);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    F[i] = (T)((double)F[i] + f * (double)e[i]);
}

// max |k^|^2 over the octant (it covers every value of |k^| by symmetry):
// per-block maxima, then the last block takes the maximum of those.
__global__ void k_smax(const double2* __restrict__ oct, long long n, double* part, uint32_t* ticket, double* out) {
  __shared__ double red[NT];
  __shared__ int last;
  double m = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const double2 k = oct[i];
    m = fmax(m, k.x * k.x + k.y * k.y);
  }
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = red[0];
    __threadfence();
    last = atomicAdd(ticket, 1u) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  m = 0.0;
  for (int k = threadIdx.x; k < (int)gridDim.x; k += NT)
    m = fmax(m, __hip_atomic_load(&part[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *out = red[0];
    *ticket = 0u;
  }
}

}  // namespace

// ============================================================ context
struct fr3d_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  std::string err;
  bool has_kernel = false, has_data = false;
  fr3d_geom g{};
  int px = 0, py = 0, pz = 0, kxn = 0;
  double D = 0;
  size_t esz = 4;  // sizeof(T)
  double smax = 0;
  double delta = 0;
  // device buffers
  double2* oct = nullptr;
  void* spec = nullptr;
  void* work = nullptr;
  size_t spec_bytes = 0, work_bytes = 0;
  Ctrl* ctrl = nullptr;
  Ctrl* ctrl_host = nullptr;  // pinned
  uint32_t* tickets = nullptr;
  double* bins_part = nullptr;
  size_t bins_part_n = 0;
  double2* norm_part = nullptr;
  size_t norm_part_n = 0;
  double* energy = nullptr;
  float* feat = nullptr;
  double* scal = nullptr;     // small FP64 scratch (norms, s_max)
  double* scal_host = nullptr;  // pinned
  std::map<int, void*> tw32, tw64;
  // timing
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev[6];
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_pool;
  double acc_ms[6] = {0, 0, 0, 0, 0, 0};
  long long cnt[6] = {0, 0, 0, 0, 0, 0};
};

namespace {

fr3d_status fail(fr3d_ctx* c, fr3d_status s, const char* fmt, ...) {
  if (c) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    c->err = buf;
  }
  return s;
}

#define HIPCHK(c, call)                                                                       \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail((c), e_ == hipErrorOutOfMemory ? FR3D_E_NOMEM : FR3D_E_DEVICE, "%s: %s (%s:%d)", \
                  #call, hipGetErrorString(e_), __FILE__, __LINE__);                          \
  } while (0)

template <typename P> void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}

void free_geometry_buffers(fr3d_ctx* c) {
  dfree(c->oct);
  dfree(c->spec);
  dfree(c->work);
  dfree(c->bins_part);
  dfree(c->norm_part);
  for (auto& kv : c->tw32) (void)hipFree(kv.second);
  for (auto& kv : c->tw64) (void)hipFree(kv.second);
  c->tw32.clear();
  c->tw64.clear();
  c->has_kernel = c->has_data = false;
}

// e^{-2 pi i m/P}: the angle is formed and evaluated in extended precision
// (x87 long double) and rounded once to double; multiples of pi/4 are exact.
void twiddles(int P, std::vector<double>& re, std::vector<double>& im) {
  re.resize(P);
  im.resize(P);
  const long double two_pi = 6.283185307179586476925286766559005768L;
  for (int m = 0; m < P; ++m) {
    const long double a = two_pi * (long double)m / (long double)P;
    re[m] = (double)cosl(a);
    im[m] = (double)-sinl(a);
  }
  for (int m = 0; m < P; ++m) {
    if ((8LL * m) % P) continue;
    const int o = (int)((8LL * m) / P);
    const double r = 0.70710678118654752440;
    const double cr[8] = {1, r, 0, -r, -1, -r, 0, r};
    const double ci[8] = {0, -r, -1, -r, 0, r, 1, r};
    re[m] = cr[o];
    im[m] = ci[o];
  }
}

fr3d_status get_twiddles(fr3d_ctx* c, int P, bool dbl, void** out) {
  auto& map = dbl ? c->tw64 : c->tw32;
  auto it = map.find(P);
  if (it != map.end()) { *out = it->second; return FR3D_OK; }
  std::vector<double> re, im;
  twiddles(P, re, im);
  void* d = nullptr;
  if (dbl) {
    std::vector<double2> h(P);
    for (int m = 0; m < P; ++m) h[m] = make_double2(re[m], im[m]);
    HIPCHK(c, hipMalloc(&d, sizeof(double2) * P));
    HIPCHK(c, hipMemcpy(d, h.data(), sizeof(double2) * P, hipMemcpyHostToDevice));
  } else {
    std::vector<float2> h(P);
    for (int m = 0; m < P; ++m) h[m] = make_float2((float)re[m], (float)im[m]);
    HIPCHK(c, hipMalloc(&d, sizeof(float2) * P));
    HIPCHK(c, hipMemcpy(d, h.data(), sizeof(float2) * P, hipMemcpyHostToDevice));
  }
  map[P] = d;
  *out = d;
  return FR3D_OK;
}

fr3d_status ensure(fr3d_ctx* c, void** p, size_t& have, size_t need) {
  if (have >= need && *p) return FR3D_OK;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  have = 0;
  HIPCHK(c, hipMalloc(p, need));
  have = need;
  return FR3D_OK;
}

// --------------------------------------------------------------- timing
// With timing on, each pass kernel is launched with an event pair recorded at
// its own start and end.
Launch mkL(fr3d_ctx* c, int pass) {
  Launch L{c->stream, nullptr, nullptr};
  if (!c->timing) return L;
  std::pair<hipEvent_t, hipEvent_t> p;
  if (!c->ev_pool.empty()) { p = c->ev_pool.back(); c->ev_pool.pop_back(); }
  else if (hipEventCreate(&p.first) != hipSuccess || hipEventCreate(&p.second) != hipSuccess) return L;
  c->ev[pass].push_back(p);
  L.e0 = p.first;
  L.e1 = p.second;
  return L;
}

// Accumulate recorded pass times.  keep_inv >= 0 counts only the first
// keep_inv launches of each inverse pass (the later launches of a search
// return at once after the search has finished).
void tcollect(fr3d_ctx* c, long long keep_inv = -1) {
  (void)hipStreamSynchronize(c->stream);
  for (int p = 0; p < 6; ++p) {
    const size_t lim = (keep_inv >= 0 && p >= 3) ? std::min<size_t>(c->ev[p].size(), (size_t)keep_inv) : c->ev[p].size();
    for (size_t i = 0; i < c->ev[p].size(); ++i) {
      auto& e = c->ev[p][i];
      float ms = 0;
      if (i < lim && hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) { c->acc_ms[p] += ms; c->cnt[p] += 1; }
      c->ev_pool.push_back(e);
    }
    c->ev[p].clear();
  }
}

// --------------------------------------------------------------- geometry
int gap_default(int nz, int q) {
  if (q < 0) return nz + (nz + 3) / 4;
  return nz + (q + 1) * ((nz + 7) / 8);
}

BinGeom bin_geom(int px, int py, int pz) {
  BinGeom b;
  b.px = px; b.py = py; b.pz = pz;
  long long l = std::lcm((long long)px, std::lcm((long long)py, (long long)pz));
  b.fx = (l / px) * (l / px);
  b.fy = (l / py) * (l / py);
  b.fz = (l / pz) * (l / pz);
  b.L3 = 3 * l * l;
  return b;
}

template <typename T> struct Bufs {
  c2<T>* S;
  c2<T>* A;
  c2<T>* B;
  c4<T>* W1;
  c4<T>* W2;
};

template <typename T> Bufs<T> bufs(fr3d_ctx* c) {
  Bufs<T> b;
  const size_t nA = (size_t)c->kxn * c->g.nz * c->g.ny;
  const size_t nB = (size_t)c->kxn * c->g.nz * c->py;
  b.S = (c2<T>*)c->spec;
  b.W1 = (c4<T>*)c->work;
  b.W2 = b.W1 + nB;
  b.A = (c2<T>*)c->work;
  b.B = b.A + nA;
  return b;
}

FwdArgs fwd_args(fr3d_ctx* c, bool kernel) {
  FwdArgs a{};
  a.nz_in = kernel ? c->pz : c->g.nz;
  a.ny_in = kernel ? c->py : c->g.ny;
  a.kx_n = c->kxn;
  a.py = c->py;
  a.pz = c->pz;
  a.h = c->g.h;
  a.D = c->D;
  a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz;
  a.kind = c->g.kind;
  a.bg = bin_geom(c->px, c->py, c->pz);
  a.bins_part = c->bins_part;
  a.bins_out = c->energy;
  a.feat_out = c->feat;
  a.ticket = c->tickets + 0;
  a.delta = c->delta;
  return a;
}

InvArgs inv_args(fr3d_ctx* c, bool search) {
  InvArgs a{};
  a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz;
  a.kx_n = c->kxn; a.py = c->py; a.pz = c->pz;
  a.scale = 1.0 / ((double)c->px * c->py * c->pz);
  a.oct = c->oct;
  a.ctrl = search ? c->ctrl : nullptr;
  a.norm_part = c->norm_part;
  return a;
}

#define LCHK(c, call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail((c), FR3D_E_DEVICE, "launch %s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

template <typename T> fr3d_status forward_data(fr3d_ctx* c, const T* F) {
  void *twx, *twy, *twz;
  const bool dbl = sizeof(T) == 8;
  if (get_twiddles(c, c->px, dbl, &twx) || get_twiddles(c, c->py, dbl, &twy) || get_twiddles(c, c->pz, dbl, &twz))
    return FR3D_E_DEVICE;
  Bufs<T> b = bufs<T>(c);
  FwdArgs a = fwd_args(c, false);
  LCHK(c, launch_fx<T>(c->px, false, F, b.A, a, (const c2<T>*)twx, mkL(c, 0)));
  LCHK(c, launch_fy<T>(c->py, true, b.A, b.B, a, (const c2<T>*)twy, mkL(c, 1)));
  LCHK(c, launch_fz<T>(c->pz, 0, b.B, b.S, a, (const c2<T>*)twz, mkL(c, 2)));
  return FR3D_OK;
}

template <typename T> fr3d_status inverse(fr3d_ctx* c, int mode, T* out) {
  void *twx, *twy, *twz;
  const bool dbl = sizeof(T) == 8;
  if (get_twiddles(c, c->px, dbl, &twx) || get_twiddles(c, c->py, dbl, &twy) || get_twiddles(c, c->pz, dbl, &twz))
    return FR3D_E_DEVICE;
  Bufs<T> b = bufs<T>(c);
  InvArgs a = inv_args(c, mode == 0);
  LCHK(c, launch_iz<T>(c->pz, mode, b.S, b.W1, a, (const c2<T>*)twz, mkL(c, 3)));
  LCHK(c, launch_iy<T>(c->py, b.W1, b.W2, a, (const c2<T>*)twy, mkL(c, 4)));
  LCHK(c, launch_ix<T>(c->px, mode, b.W2, out, a, (const c2<T>*)twx, mkL(c, 5)));
  return FR3D_OK;
}

fr3d_status launch_ctrl(fr3d_ctx* c, const Ctrl& v) {
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(1), 0, c->stream, c->ctrl, v);
  LCHK(c, hipGetLastError());
  return FR3D_OK;
}

Ctrl ctrl_base(fr3d_ctx* c) {
  Ctrl v{};
  v.a_scale = c->g.alpha_relative ? c->smax : 1.0;
  v.delta = c->delta;
  v.tau = 1.0;
  v.h_op = 0.0;
  v.mu = 0.0;
  v.tol = 1e-3;
  v.acc_lo = 0.9;
  v.acc_hi = 1.1;
  v.lo = -8.0;
  v.hi = 0.0;
  v.max_steps = 40;
  v.active = 1;
  return v;
}

fr3d_status read_ctrl(fr3d_ctx* c) {
  HIPCHK(c, hipMemcpyAsync(c->ctrl_host, c->ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  return FR3D_OK;
}

void fill_report(fr3d_ctx* c, fr3d_report* r) {
  const Ctrl& h = *c->ctrl_host;
  r->alpha = std::pow(10.0, h.t);
  r->residual = std::sqrt(h.r2);
  r->zeta_norm = std::sqrt(h.z2);
  r->delta = h.delta;
  r->target = h.target;
  r->n_evals = h.n_evals;
  r->flags = h.flags;
}

bool need(fr3d_ctx* c, bool kernel, bool data) {
  if (kernel && !c->has_kernel) { fail(c, FR3D_E_STATE, "no kernel loaded"); return false; }
  if (data && !c->has_data) { fail(c, FR3D_E_STATE, "no data set"); return false; }
  return true;
}

long long ncells(fr3d_ctx* c) { return (long long)c->g.nx * c->g.ny * c->g.nz; }

int env_int(const char* name, int dflt) {
  const char* s = std::getenv(name);
  return s ? std::atoi(s) : dflt;
}

}  // namespace

// ============================================================ C-ABI
extern "C" {

void fr3d_dp_opts_default(fr3d_dp_opts* o) {
  if (!o) return;
  o->log10_alpha_lo = -8.0;
  o->log10_alpha_hi = 0.0;
  o->max_steps = 40;
  o->tol = 1e-3;
  o->accept_lo = 0.9;
  o->accept_hi = 1.1;
  o->tau = 1.0;
  o->h_op = 0.0;
  o->mu = 0.0;
  o->use_predictor = 0;
}

const char* fr3d_status_string(fr3d_status s) {
  switch (s) {
    case FR3D_OK: return "ok";
    case FR3D_E_INVALID: return "invalid argument";
    case FR3D_E_STATE: return "call out of order";
    case FR3D_E_NOMEM: return "device allocation failed";
    case FR3D_E_DEVICE: return "device error";
  }
  return "unknown status";
}

const char* fr3d_last_error(const fr3d_ctx* c) { return c ? c->err.c_str() : "null context"; }

fr3d_status fr3d_create(fr3d_ctx** out, int32_t device, void* stream) {
  if (!out) return FR3D_E_INVALID;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || n <= 0 || device < 0 || device >= n) return FR3D_E_DEVICE;
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return FR3D_E_DEVICE;
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return FR3D_E_DEVICE;
  if (hipSetDevice(device) != hipSuccess) return FR3D_E_DEVICE;
  fr3d_ctx* c = new (std::nothrow) fr3d_ctx;
  if (!c) return FR3D_E_NOMEM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  bool ok = hipMalloc(&c->ctrl, sizeof(Ctrl)) == hipSuccess &&
            hipHostMalloc(&c->ctrl_host, sizeof(Ctrl), hipHostMallocDefault) == hipSuccess &&
            hipMalloc(&c->tickets, 16 * sizeof(uint32_t)) == hipSuccess &&
            hipMalloc(&c->energy, 64 * sizeof(double)) == hipSuccess &&
            hipMalloc(&c->feat, 65 * sizeof(float)) == hipSuccess &&
            hipMalloc(&c->scal, 16 * sizeof(double)) == hipSuccess &&
            hipHostMalloc(&c->scal_host, 16 * sizeof(double), hipHostMallocDefault) == hipSuccess &&
            hipMemset(c->tickets, 0, 16 * sizeof(uint32_t)) == hipSuccess &&
            hipMemset(c->ctrl, 0, sizeof(Ctrl)) == hipSuccess && hipDeviceSynchronize() == hipSuccess;
  if (!ok) {
    fr3d_destroy(c);
    return FR3D_E_NOMEM;
  }
  *out = c;
  return FR3D_OK;
}

fr3d_status fr3d_destroy(fr3d_ctx* c) {
  if (!c) return FR3D_E_INVALID;
  (void)hipSetDevice(c->device);
  if (c->stream) (void)hipStreamSynchronize(c->stream);
  else (void)hipDeviceSynchronize();
  free_geometry_buffers(c);
  dfree(c->ctrl);
  if (c->ctrl_host) (void)hipHostFree(c->ctrl_host);
  if (c->scal_host) (void)hipHostFree(c->scal_host);
  dfree(c->tickets);
  dfree(c->energy);
  dfree(c->feat);
  dfree(c->scal);
  for (int p = 0; p < 6; ++p)
    for (auto& e : c->ev[p]) c->ev_pool.push_back(e);
  for (auto& e : c->ev_pool) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  delete c;
  return FR3D_OK;
}

fr3d_status fr3d_set_stream(fr3d_ctx* c, void* stream) {
  if (!c) return FR3D_E_INVALID;
  c->stream = (hipStream_t)stream;
  return FR3D_OK;
}

fr3d_status fr3d_load_kernel(fr3d_ctx* c, const fr3d_geom* g) {
  if (!c) return FR3D_E_INVALID;
  if (!g) return fail(c, FR3D_E_INVALID, "geom is null");
  if (g->nx < 2 || g->ny < 2 || g->nz < 2) return fail(c, FR3D_E_INVALID, "grid extents must be >= 2");
  if (!supported_length(2 * g->nx) || !supported_length(2 * g->ny) || !supported_length(2 * g->nz))
    return fail(c, FR3D_E_INVALID, "2n per axis must be one of the compiled lengths (2^a 3^b, <= 512)");
  if (!(g->h > 0) || !std::isfinite(g->h)) return fail(c, FR3D_E_INVALID, "h must be finite and > 0");
  if (g->kind != 0 && g->kind != 1) return fail(c, FR3D_E_INVALID, "kind must be 0 or 1");
  if (g->precision != 32 && g->precision != 64) return fail(c, FR3D_E_INVALID, "precision must be 32 or 64");
  if (!std::isfinite(g->D)) return fail(c, FR3D_E_INVALID, "D must be finite");
  if (g->alpha_relative != 0 && g->alpha_relative != 1) return fail(c, FR3D_E_INVALID, "alpha_relative must be 0 or 1");
  const double D = g->D > 0 ? g->D : (double)gap_default(g->nz, g->q);
  if (D < g->nz) return fail(c, FR3D_E_INVALID, "D must be >= nz (R and Y disjoint)");
  HIPCHK(c, hipSetDevice(c->device));
  HIPCHK(c, c->stream ? hipStreamSynchronize(c->stream) : hipDeviceSynchronize());
  free_geometry_buffers(c);
  c->g = *g;
  c->D = D;
  c->px = 2 * g->nx; c->py = 2 * g->ny; c->pz = 2 * g->nz;
  c->kxn = c->px / 2 + 1;
  c->esz = g->precision == 64 ? 8 : 4;
  const size_t kxn = c->kxn;
  const size_t nS = kxn * c->pz * c->py;
  const size_t nA = kxn * g->nz * g->ny, nB = kxn * g->nz * c->py;
  c->spec_bytes = nS * 2 * c->esz;
  c->work_bytes = (nA + nB) * 4 * c->esz;  // W1 + W2 (pairs) cover A + B
  const size_t noct = kxn * (c->pz / 2 + 1) * (c->py / 2 + 1);
  HIPCHK(c, hipMalloc(&c->oct, noct * sizeof(double2)));
  HIPCHK(c, hipMalloc(&c->spec, c->spec_bytes));
  HIPCHK(c, hipMalloc(&c->work, c->work_bytes));
  // partial-sum buffers sized for the largest grid of either precision
  c->bins_part_n = (size_t)kxn * c->py;  // >= blocks of the z pass
  HIPCHK(c, hipMalloc(&c->bins_part, c->bins_part_n * 64 * sizeof(double)));
  c->norm_part_n = (size_t)g->nz * g->ny;  // >= blocks of the x pass
  HIPCHK(c, hipMalloc(&c->norm_part, c->norm_part_n * sizeof(double2)));

  // kernel spectrum in FP64 through full (unpruned) passes; temporaries freed after
  double2 *Ak = nullptr, *Bk = nullptr;
  HIPCHK(c, hipMalloc(&Ak, nS * sizeof(double2)));
  hipError_t e2 = hipMalloc(&Bk, nS * sizeof(double2));
  if (e2 != hipSuccess) { (void)hipFree(Ak); return fail(c, FR3D_E_NOMEM, "kernel spectrum workspace: %s", hipGetErrorString(e2)); }
  void *twx, *twy, *twz;
  fr3d_status st = FR3D_OK;
  if ((st = get_twiddles(c, c->px, true, &twx)) || (st = get_twiddles(c, c->py, true, &twy)) ||
      (st = get_twiddles(c, c->pz, true, &twz))) {
    (void)hipFree(Ak); (void)hipFree(Bk);
    return st;
  }
  FwdArgs a = fwd_args(c, true);
  const Launch L{c->stream, nullptr, nullptr};
  hipError_t le = launch_fx<double>(c->px, true, nullptr, Ak, a, (const double2*)twx, L);
  if (le == hipSuccess) le = launch_fy<double>(c->py, false, Ak, Bk, a, (const double2*)twy, L);
  if (le == hipSuccess) le = launch_fz<double>(c->pz, 1, Bk, c->oct, a, (const double2*)twz, L);
  if (le == hipSuccess) {
    const unsigned nb = (unsigned)std::min<long long>(((long long)noct + NT - 1) / NT, 1024);
    hipLaunchKernelGGL(k_smax, dim3(nb), dim3(NT), 0, c->stream, c->oct, (long long)noct, (double*)Ak,
                       c->tickets + 3, c->scal);
    le = hipGetLastError();
  }
  if (le == hipSuccess) le = hipMemcpyAsync(c->scal_host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream);
  if (le == hipSuccess) le = hipStreamSynchronize(c->stream);
  (void)hipFree(Ak);
  (void)hipFree(Bk);
  if (le != hipSuccess) return fail(c, FR3D_E_DEVICE, "kernel spectrum: %s", hipGetErrorString(le));
  c->smax = c->scal_host[0];
  if (!(c->smax > 0) || !std::isfinite(c->smax)) return fail(c, FR3D_E_DEVICE, "kernel spectrum has no energy");
  // precision twiddles for the data passes
  const bool dbl = c->esz == 8;
  if ((st = get_twiddles(c, c->px, dbl, &twx)) || (st = get_twiddles(c, c->py, dbl, &twy)) ||
      (st = get_twiddles(c, c->pz, dbl, &twz)))
    return st;
  c->has_kernel = true;
  c->has_data = false;
  return FR3D_OK;
}

fr3d_status fr3d_set_data(fr3d_ctx* c, const void* F, double delta) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!F) return fail(c, FR3D_E_INVALID, "F is null");
  if (!(delta >= 0) || !std::isfinite(delta)) return fail(c, FR3D_E_INVALID, "delta must be finite and >= 0");
  c->delta = delta;
  fr3d_status s = c->esz == 8 ? forward_data<double>(c, (const double*)F) : forward_data<float>(c, (const float*)F);
  if (s) return s;
  c->has_data = true;
  return FR3D_OK;
}

static fr3d_status run_search(fr3d_ctx* c, const Ctrl& init, int max_evals, void* zeta, fr3d_report* rep) {
  if (c->timing) tcollect(c);
  fr3d_status s = launch_ctrl(c, init);
  if (s) return s;
  const int chunk = std::max(1, env_int("FR3D_EVAL_CHUNK", 4));
  int launched = 0;
  for (;;) {
    const int k = std::min(chunk, max_evals - launched);
    for (int i = 0; i < k; ++i) {
      s = c->esz == 8 ? inverse<double>(c, 0, (double*)zeta) : inverse<float>(c, 0, (float*)zeta);
      if (s) return s;
    }
    launched += k;
    if ((s = read_ctrl(c))) return s;
    if (!c->ctrl_host->active || launched >= max_evals) break;
  }
  if (c->timing) tcollect(c, c->ctrl_host->n_evals);
  if (c->ctrl_host->active) return fail(c, FR3D_E_DEVICE, "alpha search did not finish in %d evaluations", max_evals);
  if (rep) fill_report(c, rep);
  return FR3D_OK;
}

fr3d_status fr3d_solve_alpha(fr3d_ctx* c, double alpha_rel, void* zeta, fr3d_report* rep) {
  // alpha_rel is in the context's alpha units (geom.alpha_relative)
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, true)) return FR3D_E_STATE;
  if (!zeta) return fail(c, FR3D_E_INVALID, "zeta is null");
  if (!(alpha_rel > 0) || !std::isfinite(alpha_rel)) return fail(c, FR3D_E_INVALID, "alpha must be finite and > 0");
  Ctrl v = ctrl_base(c);
  v.state = ST_FIXED;
  v.t = std::log10(alpha_rel);
  v.alpha_abs = alpha_rel * v.a_scale;
  return run_search(c, v, 1, zeta, rep);
}

fr3d_status fr3d_solve_discrepancy(fr3d_ctx* c, const fr3d_dp_opts* o, void* zeta, fr3d_report* rep) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, true)) return FR3D_E_STATE;
  if (!zeta) return fail(c, FR3D_E_INVALID, "zeta is null");
  fr3d_dp_opts d;
  fr3d_dp_opts_default(&d);
  if (o) d = *o;
  if (!(d.log10_alpha_lo < d.log10_alpha_hi) || !std::isfinite(d.log10_alpha_lo) || !std::isfinite(d.log10_alpha_hi) ||
      d.max_steps < 0 || d.max_steps > 200 || !(d.tol >= 0) || !(d.tau > 0) || !(d.h_op >= 0) || !(d.mu >= 0))
    return fail(c, FR3D_E_INVALID, "bad search options");
  if (d.use_predictor) return fail(c, FR3D_E_STATE, "no predictor loaded");
  Ctrl v = ctrl_base(c);
  v.lo = d.log10_alpha_lo;
  v.hi = d.log10_alpha_hi;
  v.max_steps = d.max_steps;
  v.tol = d.tol;
  v.acc_lo = d.accept_lo;
  v.acc_hi = d.accept_hi;
  v.tau = d.tau;
  v.h_op = d.h_op;
  v.mu = d.mu;
  v.state = ST_HI;
  v.t = v.hi;
  v.alpha_abs = std::pow(10.0, v.hi) * v.a_scale;
  return run_search(c, v, 2 + d.max_steps + 1, zeta, rep);
}

fr3d_status fr3d_recover_c(fr3d_ctx* c, const void* zeta, const void* V0, double c0, void* cout, int64_t* ncl) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!zeta || !V0 || !cout) return fail(c, FR3D_E_INVALID, "null array");
  if (!(c0 > 0) || !std::isfinite(c0)) return fail(c, FR3D_E_INVALID, "c0 must be finite and > 0");
  const long long n = ncells(c);
  double* part = (double*)c->norm_part;  // >= 2 nz ny doubles
  const double ic2 = 1.0 / (c0 * c0), fl = 1e-6 / (c0 * c0);
  const unsigned nb = (unsigned)std::min<long long>((n + NT - 1) / NT, 2048);
  if (c->esz == 8)
    hipLaunchKernelGGL(k_recover<double>, dim3(nb), dim3(NT), 0, c->stream, (const double*)zeta, (const double*)V0,
                       ic2, fl, (double*)cout, n, part);
  else
    hipLaunchKernelGGL(k_recover<float>, dim3(nb), dim3(NT), 0, c->stream, (const float*)zeta, (const float*)V0, ic2,
                       fl, (float*)cout, n, part);
  LCHK(c, hipGetLastError());
  if (ncl) {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(NT), 0, c->stream, (const double*)part, (int)nb, 1, 1, c->scal);
    LCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(c->scal_host, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    *ncl = (int64_t)c->scal_host[0];
  }
  return FR3D_OK;
}

fr3d_status fr3d_source_potential(fr3d_ctx* c, double A0, void* V0) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!V0) return fail(c, FR3D_E_INVALID, "V0 is null");
  if (!std::isfinite(A0)) return fail(c, FR3D_E_INVALID, "A0 must be finite");
  Sources s;
  const double G = c->D - c->g.nz, h = c->g.h;
  const double cx = c->g.nx / 2.0, cy = c->g.ny / 2.0, ax = 0.4 * c->g.nx, ay = 0.4 * c->g.ny;
  const double lx[5] = {cx, cx - ax, cx + ax, cx, cx}, ly[5] = {cy, cy, cy, cy - ay, cy + ay};
  const double hz[2] = {c->g.nz + G / 4.0, c->g.nz + 3.0 * G / 4.0};
  for (int k = 0; k < 2; ++k)
    for (int l = 0; l < 5; ++l) {
      s.x[5 * k + l] = lx[l] * h;
      s.y[5 * k + l] = ly[l] * h;
      s.z[5 * k + l] = hz[k] * h;
    }
  const long long n = ncells(c);
  dim3 grid((unsigned)std::min<long long>((n + 255) / 256, 4096));
  if (c->esz == 8)
    hipLaunchKernelGGL(k_v0<double>, grid, dim3(256), 0, c->stream, (double*)V0, c->g.nx, c->g.ny, c->g.nz, h, A0, s);
  else
    hipLaunchKernelGGL(k_v0<float>, grid, dim3(256), 0, c->stream, (float*)V0, c->g.nx, c->g.ny, c->g.nz, h, A0, s);
  LCHK(c, hipGetLastError());
  return FR3D_OK;
}

fr3d_status fr3d_apply_operator(fr3d_ctx* c, const void* zeta, void* F) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!zeta || !F) return fail(c, FR3D_E_INVALID, "null array");
  fr3d_status s;
  if (c->esz == 8) {
    if ((s = forward_data<double>(c, (const double*)zeta))) return s;
    s = inverse<double>(c, 1, (double*)F);
  } else {
    if ((s = forward_data<float>(c, (const float*)zeta))) return s;
    s = inverse<float>(c, 1, (float*)F);
  }
  c->has_data = false;  // the spectrum buffer now holds zeta's transform
  return s;
}

fr3d_status fr3d_add_noise(fr3d_ctx* c, void* F, const void* e, double delta_rel, double* delta) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!F || !e) return fail(c, FR3D_E_INVALID, "null array");
  if (!(delta_rel >= 0) || !std::isfinite(delta_rel)) return fail(c, FR3D_E_INVALID, "delta_rel must be >= 0");
  const long long n = ncells(c);
  const unsigned nb = (unsigned)std::min<long long>((n + NT - 1) / NT, 1024);
  double* nrm = c->scal + 2;
  double* part = (double*)c->norm_part;
  if (c->esz == 8)
    hipLaunchKernelGGL(k_norms2<double>, dim3(nb), dim3(NT), 0, c->stream, (const double*)F, (const double*)e, n, part);
  else
    hipLaunchKernelGGL(k_norms2<float>, dim3(nb), dim3(NT), 0, c->stream, (const float*)F, (const float*)e, n, part);
  LCHK(c, hipGetLastError());
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(NT), 0, c->stream, (const double*)part, (int)nb, 2, 2, nrm);
  LCHK(c, hipGetLastError());
  dim3 grid((unsigned)std::min<long long>((n + 255) / 256, 4096));
  if (c->esz == 8)
    hipLaunchKernelGGL(k_add_noise<double>, grid, dim3(256), 0, c->stream, (double*)F, (const double*)e, n, delta_rel, nrm);
  else
    hipLaunchKernelGGL(k_add_noise<float>, grid, dim3(256), 0, c->stream, (float*)F, (const float*)e, n, delta_rel, nrm);
  LCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(c->scal_host, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  HIPCHK(c, hipStreamSynchronize(c->stream));
  if (delta) *delta = delta_rel * std::sqrt(c->scal_host[0]);
  return FR3D_OK;
}

fr3d_status fr3d_get_octant(fr3d_ctx* c, void* out, int64_t bytes) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  const size_t n = (size_t)c->kxn * (c->pz / 2 + 1) * (c->py / 2 + 1) * sizeof(double2);
  if (!out || bytes < (int64_t)n) return fail(c, FR3D_E_INVALID, "need %zu bytes", n);
  HIPCHK(c, hipMemcpyAsync(out, c->oct, n, hipMemcpyDeviceToDevice, c->stream));
  return FR3D_OK;
}

fr3d_status fr3d_get_data_spectrum(fr3d_ctx* c, void* out, int64_t bytes) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!out || bytes < (int64_t)c->spec_bytes) return fail(c, FR3D_E_INVALID, "need %zu bytes", c->spec_bytes);
  HIPCHK(c, hipMemcpyAsync(out, c->spec, c->spec_bytes, hipMemcpyDeviceToDevice, c->stream));
  return FR3D_OK;
}

fr3d_status fr3d_get_features(fr3d_ctx* c, float* feat, double* energy) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, true)) return FR3D_E_STATE;
  if (feat) HIPCHK(c, hipMemcpyAsync(feat, c->feat, 65 * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
  if (energy) HIPCHK(c, hipMemcpyAsync(energy, c->energy, 64 * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
  return FR3D_OK;
}

fr3d_status fr3d_get_smax(fr3d_ctx* c, double* smax) {
  if (!c || !smax) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  *smax = c->smax;
  return FR3D_OK;
}

fr3d_status fr3d_set_timing(fr3d_ctx* c, int32_t enable) {
  if (!c) return FR3D_E_INVALID;
  if (c->timing && !enable) tcollect(c);
  c->timing = enable != 0;
  return FR3D_OK;
}

fr3d_status fr3d_get_timing(fr3d_ctx* c, int32_t pass, double* total_ms, int64_t* launches) {
  if (!c || pass < 0 || pass > 5) return FR3D_E_INVALID;
  tcollect(c);
  if (total_ms) *total_ms = c->acc_ms[pass];
  if (launches) *launches = c->cnt[pass];
  c->acc_ms[pass] = 0;
  c->cnt[pass] = 0;
  return FR3D_OK;
}

}  // extern "C"
