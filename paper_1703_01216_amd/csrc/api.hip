// C-ABI of the solver (declared in include/fr3d.h): context, lanes,
// kernel spectrum, data transform, alpha evaluations and search, batch
// scheduler, recovery, source potential, forward operator, noise and the
// alpha predictor.
//
// A context holds one geometry: the FP64 kernel-spectrum octant and the
// twiddle tables, shared read-only by its lanes.  A lane holds everything one
// solve in flight needs: a stream, the data spectrum, the inverse-pass
// workspaces, a device control block and its pinned host mirror.  Lane 0
// runs on the caller's stream and serves the single-solve calls; the batch
// call keeps every lane busy with its own instance.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <numeric>
#include <string>
#include <algorithm>
#include <thread>
#include <vector>

#include "../../include/fr3d.h"
#include "control.hpp"
#include "layered.hpp"
#include "mlp.hpp"
#include "passes.hpp"

using namespace fr3d;

// ============================================================ small kernels
namespace {

__global__ void k_ctrl_init(Ctrl* c, Ctrl v) {
  *c = v;
  if (v.state == ST_KARY) ctrl_kary_points(c);  // first step's candidates
}

// The report of a search, written on the device (the _dev solves).
__global__ void k_report(const Ctrl* c, fr3d_report* r) {
  fr3d_report o;
  o.alpha = pow(10.0, c->t);
  o.residual = sqrt(c->r2);
  o.zeta_norm = sqrt(c->z2);
  o.delta = c->delta;
  o.target = c->target;
  o.n_evals = c->n_evals;
  o.flags = c->flags | (c->active ? FR3D_UNFINISHED : 0);
  o.n_clamped = -1;
  o.residual_full_box = c->r2_full >= 0 ? sqrt(c->r2_full) : -1.0;
  *r = o;
}

// Recovery (Algorithm 1, step 4): xi = zeta / V0 and c = (1/c0^2 - xi)^(-1/2)
// with the argument clamped at 1e-6/c0^2; per-block counts of clamped cells.
// Grid-stride over the cells, the loads of U strides issued together (one
// memory round trip per U cells of a thread; cells visited in the same order).
template <typename T>
__global__ void k_recover(const T* __restrict__ zeta, const T* __restrict__ V0, double inv_c02, double floor_,
                          T* __restrict__ c, long long n, double* part) {
  constexpr int U = 4;
  __shared__ double red[NT / 64];
  double cl = 0.0;
  const long long st = (long long)gridDim.x * NT;
  for (long long i0 = (long long)blockIdx.x * NT + threadIdx.x; i0 < n; i0 += U * st) {
    T zv[U], vv[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + u * st;
      if (i < n) {
        zv[u] = zeta[i];
        vv[u] = V0[i];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const long long i = i0 + u * st;
      if (i < n) {
        const double xi = (double)zv[u] / (double)vv[u];
        double arg = inv_c02 - xi;
        if (arg < floor_) { arg = floor_; cl += 1.0; }
        c[i] = (T)(1.0 / sqrt(arg));
      }
    }
  }
  cl = block_sum<NT>(cl, red);
  if (threadIdx.x == 0) part[blockIdx.x] = cl;
}

// The clamped-cell count: the sum of k_recover's nblk partials in a fixed
// order (one workgroup), as an integer (every partial is a whole number
// below 2^53, so the FP64 sum is exact).
__global__ void k_clamp_count(const double* __restrict__ part, int nblk, int64_t* out) {
  __shared__ double red[NT / 64];
  double s = strided_sum<double>(part, threadIdx.x, nblk, NT);
  s = block_sum<NT>(s, red);
  if (threadIdx.x == 0) *out = (int64_t)s;
}

// out[j] = sum over k < nblk of part[k*stride + j] for j < nout (one workgroup, fixed order).
__global__ void k_sum_parts(const double* __restrict__ part, int nblk, int stride, int nout, double* out) {
  __shared__ double red[NT / 64];
  for (int j = 0; j < nout; ++j) {
    double s = strided_sum<double>(part + j, threadIdx.x, nblk, NT, stride);
    s = block_sum<NT>(s, red);
    if (threadIdx.x == 0) out[j] = s;
  }
}

// ---- conjugate gradients on the normal equations of the exact operator.
// Device scalars cg[]: 0 r.r, 1 p.q, 2 r.r after the step, 3 b.b, 4 x.x, 5 t.t.
template <typename T>
__global__ void k_dot_part(const T* __restrict__ a, const T* __restrict__ b, long long n, double* part) {
  __shared__ double red[NT / 64];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
    s += (double)a[i] * (double)b[i];
  s = block_sum<NT>(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// q += alpha p; partial p.q
template <typename T>
__global__ void k_cg_q(T* __restrict__ q, const T* __restrict__ p, double alpha, long long n, double* part) {
  __shared__ double red[NT / 64];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const double pv = (double)p[i];
    const T qv = (T)((double)q[i] + alpha * pv);
    q[i] = qv;
    s += pv * (double)qv;
  }
  s = block_sum<NT>(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// a = r.r / p.q;  x += a p;  r -= a q;  partial of the new r.r
template <typename T>
__global__ void k_cg_step(T* __restrict__ x, T* __restrict__ r, const T* __restrict__ p, const T* __restrict__ q,
                          long long n, const double* __restrict__ cg, double* part) {
  __shared__ double red[NT / 64];
  const double a = cg[0] / cg[1];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    x[i] = (T)((double)x[i] + a * (double)p[i]);
    const T rv = (T)((double)r[i] - a * (double)q[i]);
    r[i] = rv;
    s += (double)rv * (double)rv;
  }
  s = block_sum<NT>(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

// p = r + (r.r new / r.r) p
template <typename T>
__global__ void k_cg_dir(T* __restrict__ p, const T* __restrict__ r, long long n, const double* __restrict__ cg) {
  const double beta = cg[2] / cg[0];
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
    p[i] = (T)((double)r[i] + beta * (double)p[i]);
}

__global__ void k_cg_roll(double* cg) { cg[0] = cg[2]; }

// t -= F; partial t.t
template <typename T>
__global__ void k_sub_sq(T* __restrict__ t, const T* __restrict__ F, long long n, double* part) {
  __shared__ double red[NT / 64];
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const T v = (T)((double)t[i] - (double)F[i]);
    t[i] = v;
    s += (double)v * (double)v;
  }
  s = block_sum<NT>(s, red);
  if (threadIdx.x == 0) part[blockIdx.x] = s;
}

template <typename T> __global__ void k_fill0(T* __restrict__ x, long long n) {
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) x[i] = (T)0;
}

// V0(x) = -(A0/4 pi) sum_l 1/|x - x_l| at R's cell centres (Sec. 6 point sources).
struct Sources { double x[10], y[10], z[10]; };

template <typename T>
__global__ void k_v0(T* __restrict__ V0, int nx, int ny, int nz, double h, double hz, double A0, Sources s) {
  const long long n = (long long)nx * ny * nz;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x) {
    const int ix = (int)(i % nx), iy = (int)((i / nx) % ny), iz = (int)(i / ((long long)nx * ny));
    const double px = (ix + 0.5) * h, py = (iy + 0.5) * h, pz = (iz + 0.5) * hz;
    double acc = 0.0;
    for (int l = 0; l < 10; ++l) {
      const double dx = px - s.x[l], dy = py - s.y[l], dz = pz - s.z[l];
      acc += 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    }
    V0[i] = (T)(-(A0 / (4.0 * M_PI)) * acc);
  }
}

// Per-block sums of squares of two arrays in FP64 (part[2 blk], part[2 blk + 1]).
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

// F += e * (delta_rel ||F|| / ||e||); nrm = (||F||^2, ||e||^2).
template <typename T>
__global__ void k_add_noise(T* __restrict__ F, const T* __restrict__ e, long long n, double delta_rel,
                            const double* nrm) {
  const double f = delta_rel * sqrt(nrm[0]) / sqrt(nrm[1]);
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    F[i] = (T)((double)F[i] + f * (double)e[i]);
}

// Per-block maxima of |k^|^2 over the octant (it covers every value of |k^|).
// Kernel-spectrum levels of the predictor features: for octant entry
// (kx, mz, my) (octant layout [kx][mz][my]) the number of thresholds thr[j]
// (increasing) with |k^|^2 >= thr[j], written to level[kx][my][kz] for
// kz = mz and kz = pz - mz (rows over the whole kz range, so that a run of
// consecutive kz is a run of consecutive bytes).
struct LevelThr {
  double t[63];
};
__global__ void k_level_table(const double2* __restrict__ oct, int kxn, int oz, int oy, int pz, LevelThr thr,
                              uint8_t* __restrict__ level) {
  const long long n = (long long)kxn * oz * oy;
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT) {
    const int my = (int)(i % oy), mz = (int)((i / oy) % oz), kx = (int)(i / ((long long)oy * oz));
    const double2 k = oct[i];
    const double s = k.x * k.x + k.y * k.y;
    int lo = 0, hi = 63;  // count of thresholds <= s, by bisection
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if (thr.t[mid] <= s) lo = mid + 1;
      else hi = mid;
    }
    uint8_t* row = level + ((size_t)kx * oy + my) * pz;
    row[mz] = (uint8_t)lo;
    if (mz > 0 && mz < pz - mz) row[pz - mz] = (uint8_t)lo;
  }
}

// The octant rounded to FP32 (each component to nearest).
__global__ void k_round_octant(const double2* __restrict__ oct, long long n, float2* __restrict__ o32) {
  for (long long i = (long long)blockIdx.x * NT + threadIdx.x; i < n; i += (long long)gridDim.x * NT)
    o32[i] = make_float2((float)oct[i].x, (float)oct[i].y);
}

__global__ void k_smax_part(const double2* __restrict__ oct, long long n, double* part) {
  __shared__ double red[NT];
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
  if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Full-box residual of a single evaluation (diagnostics): the residual
// spectrum is r^ = -e(s) f^ with e the filter's residual factor (Tikhonov
// a/(s+a), iterated Tikhonov (a/(s+a))^m, truncated SVD 0 where s >= a and
// 1 elsewhere), so by Parseval ||r||^2 = (1/N) sum over the whole box of
// e^2 |f^|^2, the half spectrum kx <= Px/2 counting planes 0 < kx < Px/2
// twice.  Per-workgroup partials, then a fixed-order sum into the control
// block.
template <typename T>
__global__ void k_full_part(const c2<T>* __restrict__ S, InvArgs a) {
  __shared__ double red[NT / 64];
  if (inv_idle(a)) return;
  const double aa = a.ctrl->alpha_abs;
  const int py = a.py, pz = a.pz, oy = py / 2 + 1, oz = pz / 2 + 1;
  const int lg = spec_lg(sizeof(T), pz, py), ng = spec_ng(py, lg);
  const long long n = (long long)a.kx_n * spec_plane(pz, py, lg);  // S in storage order
  double acc = 0.0;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < n; e += (long long)gridDim.x * NT) {
    const long long row = e >> lg;  // (kx, granule, kz)
    const int ky = (int)(((row / pz) % ng) << lg) + (int)(e & ((1 << lg) - 1));
    const int kz = (int)(row % pz), kx = (int)(row / ((long long)pz * ng));
    if (ky >= py) continue;  // a partial last granule's unused columns
    const int mz = kz <= pz / 2 ? kz : pz - kz, my = ky <= py / 2 ? ky : py - ky;
    const double2 kk = a.oct[((size_t)kx * oz + mz) * oy + my];
    const double s = kk.x * kk.x + kk.y * kk.y;
    double ef;
    if (a.filt == 0) {
      ef = aa / (s + aa);
    } else if (a.filt == 1) {
      const double q = aa / (s + aa);
      ef = q;
      for (int j = 1; j < a.order; ++j) ef *= q;
    } else {
      ef = s >= aa ? 0.0 : 1.0;
    }
    const c2<T> f = S[e];
    const double w = (kx == 0 || kx == a.kx_n - 1) ? 1.0 : 2.0;
    acc += w * ef * ef * ((double)f.x * f.x + (double)f.y * f.y);
  }
  const double t = block_sum<NT>(acc, red);
  if (threadIdx.x == 0) a.full_part[blockIdx.x] = t;
}

__global__ void k_full_final(InvArgs a, int nblk) {
  __shared__ double red[NT / 64];
  if (inv_idle(a)) return;
  double s = strided_sum<double>(a.full_part, threadIdx.x, nblk, NT);
  s = block_sum<NT>(s, red);
  if (threadIdx.x == 0) a.ctrl->r2_full = s * a.scale;
}

// The data spectrum in the standard layout [Kx][Pz][Py] from its column
// granules (inspection only).
template <typename T>
__global__ void k_spec_untile(const c2<T>* __restrict__ S, c2<T>* __restrict__ out, int kxn, int pz, int py) {
  const int lg = spec_lg(sizeof(T), pz, py);
  const size_t plane = spec_plane(pz, py, lg);
  const long long n = (long long)kxn * pz * py;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < n; e += (long long)gridDim.x * NT) {
    const int ky = (int)(e % py), kz = (int)((e / py) % pz), kx = (int)(e / ((long long)py * pz));
    out[e] = S[(size_t)kx * plane + spec_off(kz, ky, pz, lg)];
  }
}

__global__ void k_max_parts(const double* __restrict__ part, int n, double* out) {
  __shared__ double red[NT];
  double m = 0.0;
  for (int k = threadIdx.x; k < n; k += NT) m = fmax(m, part[k]);
  red[threadIdx.x] = m;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + s]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = red[0];
}

}  // namespace

// ============================================================ context
struct Lane {
  hipStream_t stream = nullptr;
  bool own_stream = false;
  void* spec = nullptr;  // data spectrum S
  void* work = nullptr;  // forward A, B / inverse W1, W2
  Ctrl* ctrl = nullptr;
  Ctrl* ctrl_host = nullptr;  // pinned
  double* bins_part = nullptr;
  double2* norm_part = nullptr;
  double* energy = nullptr;
  float* feat = nullptr;
  double* scal = nullptr;       // small FP64 scratch
  double* scal_host = nullptr;  // pinned
  uint32_t* ticket = nullptr;
  void* kwork = nullptr;        // K-candidate workspaces: K slices of W1, then K of W2
  double2* knorm = nullptr;     // K-candidate norm partials
  int kcap = 0;                 // candidates the K-candidate workspaces hold
  int kmax = 0;                 // K of the lane's current search (0: not a K-candidate search)
  // while a group solve lends the lane a pooled K-candidate workspace, its own
  // (if any) is kept here
  bool kpooled = false;
  void* own_kwork = nullptr;
  double2* own_knorm = nullptr;
  int own_kcap = 0;
  bool slope_next = false;         // the next evaluation is a seed that forms the full-box slope
  hipGraphExec_t gexec = nullptr;  // captured evaluation (valid for gkmax and gsh)
  int gkmax = -1;
  int gsh[6] = {0, 0, 0, 0, 0, 0};
  hipEvent_t ev = nullptr;      // completion marker polled by the batch scheduler
  bool has_data = false;
  double delta = 0;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev[6];  // timing event pairs per pass
};

struct fr3d_ctx {
  int device = 0;
  std::string err;
  bool has_kernel = false;
  fr3d_geom g{};
  int px = 0, py = 0, pz = 0, kxn = 0;
  double D = 0;
  double hz = 1;  // vertical cell edge
  size_t esz = 4;
  double smax = 0;
  double2* oct = nullptr;
  float2* oct32 = nullptr;
  uint8_t* level = nullptr;  // kernel-spectrum level per (kx, |ky|, kz), [kx][my][kz]  // FP32 contexts: the octant rounded to FP32 once (the FP32 filter's operand)
  // per-frequency z-systems (Algorithm 1 as in Sec. 5) instead of the 3D embedding
  bool layered = false;
  double *lay_kt = nullptr, *lay_V = nullptr, *lay_lam = nullptr;
  size_t spec_bytes = 0, work_bytes = 0, bins_part_n = 0, norm_part_n = 0;
  std::map<int, void*> tw32, tw64;
  std::vector<Lane> lanes;  // lanes[0] runs on the caller's stream
  int nlanes_wanted = 1;
  int tile_sh[6] = {0, 0, 0, 0, 0, 0};  // tile-size variant per pass
  // predictor
  bool has_pred = false;
  float* pred_p = nullptr;     // parameters, FP32 master copy
  float* pred_norm = nullptr;  // 132 normalisation values
  double* pred_cal = nullptr;  // seed calibration for one geometry: 66 coefficients (device)
  bool has_cal = false;
  float* pred_m = nullptr;
  float* pred_v = nullptr;
  float* pred_g = nullptr;
  float* pred_loss = nullptr;
  void* pred_work = nullptr;
  int pred_cap = 0;
  long long pred_step = 0;
  // timing
  bool timing = false;
  int filt = 0, forder = 1;          // regularising filter and its order
  // conjugate-gradient workspace of the exact-operator solves (r, p, q, t; partials; scalars)
  void* cg_buf = nullptr;
  size_t cg_cap = 0;
  double* cg_part = nullptr;
  double* cg_dev = nullptr;
  double* cg_host = nullptr;  // pinned
  double* pf_part = nullptr;  // per-system partials of the per-frequency alpha search
  size_t pf_cap = 0;
  // K-candidate workspaces a group solve with this context first lends to the
  // lanes of all its contexts (fr3d_solve_group): a few slots, each sized for
  // the largest geometry of the group, so the memory does not grow with the
  // number of contexts
  std::vector<void*> pool_kw;
  std::vector<double2*> pool_kn;
  size_t pool_kw_bytes = 0, pool_kn_bytes = 0;
  bool graphs = false;              // replay each lane's evaluation as a captured HIP graph
  bool diag = false;                // form the full-box residual of every single evaluation
  hipStream_t cap_stream = nullptr; // stream the graphs are captured on
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

#define LCHK(c, call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess) return fail((c), FR3D_E_DEVICE, "launch %s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

template <typename P> void dfree(P*& p) {
  if (p) (void)hipFree((void*)p);
  p = nullptr;
}
template <typename P> void hfree(P*& p) {
  if (p) (void)hipHostFree((void*)p);
  p = nullptr;
}

void free_lane_geometry(Lane& L) {
  dfree(L.spec);
  dfree(L.work);
  dfree(L.bins_part);
  dfree(L.norm_part);
  if (L.kpooled) {  // a lent workspace belongs to the pool
    L.kwork = L.own_kwork;
    L.knorm = L.own_knorm;
    L.kpooled = false;
  }
  dfree(L.kwork);
  dfree(L.knorm);
  L.own_kwork = nullptr;
  L.own_knorm = nullptr;
  L.kcap = 0;
  L.kmax = 0;
  if (L.gexec) (void)hipGraphExecDestroy(L.gexec);
  L.gexec = nullptr;
  L.gkmax = -1;
  L.has_data = false;
}

void free_lane(Lane& L) {
  free_lane_geometry(L);
  dfree(L.ctrl);
  hfree(L.ctrl_host);
  dfree(L.energy);
  dfree(L.feat);
  dfree(L.scal);
  hfree(L.scal_host);
  dfree(L.ticket);
  if (L.ev) (void)hipEventDestroy(L.ev);
  L.ev = nullptr;
  if (L.own_stream && L.stream) (void)hipStreamDestroy(L.stream);
  L.stream = nullptr;
}

fr3d_status init_lane(fr3d_ctx* c, Lane& L, hipStream_t stream, bool own) {
  L.stream = stream;
  L.own_stream = own;
  HIPCHK(c, hipMalloc(&L.ctrl, sizeof(Ctrl)));
  HIPCHK(c, hipHostMalloc(&L.ctrl_host, sizeof(Ctrl), hipHostMallocDefault));
  HIPCHK(c, hipMalloc(&L.energy, 64 * sizeof(double)));
  HIPCHK(c, hipMalloc(&L.feat, 65 * sizeof(float)));
  HIPCHK(c, hipMalloc(&L.scal, 16 * sizeof(double)));
  HIPCHK(c, hipHostMalloc(&L.scal_host, 16 * sizeof(double), hipHostMallocDefault));
  HIPCHK(c, hipMalloc(&L.ticket, 4 * sizeof(uint32_t)));
  HIPCHK(c, hipMemset(L.ticket, 0, 4 * sizeof(uint32_t)));
  HIPCHK(c, hipMemset(L.ctrl, 0, sizeof(Ctrl)));
  HIPCHK(c, hipEventCreateWithFlags(&L.ev, hipEventDisableTiming));
  std::memset(L.ctrl_host, 0, sizeof(Ctrl));
  return FR3D_OK;
}

fr3d_status alloc_lane_geometry(fr3d_ctx* c, Lane& L) {
  free_lane_geometry(L);
  HIPCHK(c, hipMalloc(&L.spec, c->spec_bytes));
  HIPCHK(c, hipMalloc(&L.work, c->work_bytes));
  HIPCHK(c, hipMalloc(&L.bins_part, c->bins_part_n * 64 * sizeof(double)));
  HIPCHK(c, hipMalloc(&L.norm_part, c->norm_part_n * sizeof(double2)));
  return FR3D_OK;
}

void free_geometry(fr3d_ctx* c) {
  dfree(c->oct);
  dfree(c->oct32);
  dfree(c->level);
  dfree(c->lay_kt);
  dfree(c->lay_V);
  dfree(c->lay_lam);
  c->layered = false;
  for (auto& kv : c->tw32) (void)hipFree(kv.second);
  for (auto& kv : c->tw64) (void)hipFree(kv.second);
  c->tw32.clear();
  c->tw64.clear();
  for (auto& L : c->lanes) free_lane_geometry(L);
  c->has_kernel = false;
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

// --------------------------------------------------------------- timing
// With timing on, each pass kernel is launched with an event pair recorded at
// its own start and end.
Launch mkL(fr3d_ctx* c, Lane& L, int pass) {
  Launch r{L.stream, nullptr, nullptr, c->tile_sh[pass]};
  if (!c->timing) return r;
  std::pair<hipEvent_t, hipEvent_t> p;
  if (!c->ev_pool.empty()) { p = c->ev_pool.back(); c->ev_pool.pop_back(); }
  else if (hipEventCreate(&p.first) != hipSuccess || hipEventCreate(&p.second) != hipSuccess) return r;
  L.tev[pass].push_back(p);
  r.e0 = p.first;
  r.e1 = p.second;
  return r;
}

// Accumulate a lane's recorded pass times (its stream must be idle).
// keep_inv >= 0 counts only the first keep_inv launches of each inverse pass
// since the last collection (later launches of a search return at once).
void tcollect(fr3d_ctx* c, Lane& L, long long keep_inv = -1) {
  for (int p = 0; p < 6; ++p) {
    const size_t lim = (keep_inv >= 0 && p >= 3) ? std::min<size_t>(L.tev[p].size(), (size_t)keep_inv) : L.tev[p].size();
    for (size_t i = 0; i < L.tev[p].size(); ++i) {
      auto& e = L.tev[p][i];
      float ms = 0;
      if (i < lim && hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess) { c->acc_ms[p] += ms; c->cnt[p] += 1; }
      c->ev_pool.push_back(e);
    }
    L.tev[p].clear();
  }
}

// --------------------------------------------------------------- geometry helpers
int gap_default(int nz, int q) {
  if (q < 0) return nz + (nz + 3) / 4;
  return nz + (q + 1) * ((nz + 7) / 8);
}

BinGeom bin_geom(int px, int py, int pz) {
  BinGeom b;
  b.px = px; b.py = py; b.pz = pz;
  return b;
}

template <typename T> struct Bufs {
  c2<T>* S;
  c2<T>* A;
  c2<T>* B;
  c4<T>* W1;
  c4<T>* W2;
};

template <typename T> Bufs<T> bufs(fr3d_ctx* c, Lane& L) {
  Bufs<T> b;
  const size_t nA = (size_t)c->kxn * c->g.nz * c->g.ny;
  const size_t nB = (size_t)c->kxn * c->g.nz * c->py;
  b.S = (c2<T>*)L.spec;
  b.W1 = (c4<T>*)L.work;
  b.W2 = b.W1 + nB;
  b.A = (c2<T>*)L.work;
  b.B = b.A + nA;
  return b;
}

FwdArgs fwd_args(fr3d_ctx* c, Lane& L, bool kernel) {
  FwdArgs a{};
  a.nz_in = kernel ? c->pz : c->g.nz;
  a.ny_in = kernel ? c->py : c->g.ny;
  a.kx_n = c->kxn;
  a.py = c->py;
  a.pz = c->pz;
  a.h = c->g.h;
  a.hz = c->hz;
  a.D = c->D;
  a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz;
  a.kind = c->g.kind;
  a.bg = bin_geom(c->px, c->py, c->pz);
  a.level = c->level;
  a.bins_part = L.bins_part;
  a.bins_out = L.energy;
  a.feat_out = L.feat;
  a.ticket = L.ticket;
  a.delta = L.delta;
  return a;
}

InvArgs inv_args(fr3d_ctx* c, Lane& L, bool search) {
  InvArgs a{};
  a.nx = c->g.nx; a.ny = c->g.ny; a.nz = c->g.nz;
  a.kx_n = c->kxn; a.py = c->py; a.pz = c->pz;
  // the per-frequency path inverts a lateral (2D) transform only
  a.scale = c->layered ? 1.0 / ((double)c->px * c->py) : 1.0 / ((double)c->px * c->py * c->pz);
  a.oct = c->oct;
  a.oct32 = c->oct32;
  a.ctrl = search ? L.ctrl : nullptr;
  a.norm_part = L.norm_part;
  a.filt = c->filt;
  a.order = c->forder;
  return a;
}

template <typename T> fr3d_status forward_data(fr3d_ctx* c, Lane& L, const T* F) {
  const bool dbl = sizeof(T) == 8;
  void *twx, *twy, *twz;
  fr3d_status st;
  if ((st = get_twiddles(c, c->px, dbl, &twx)) || (st = get_twiddles(c, c->py, dbl, &twy)) ||
      (st = get_twiddles(c, c->pz, dbl, &twz)))
    return st;
  Bufs<T> b = bufs<T>(c, L);
  FwdArgs a = fwd_args(c, L, false);
  LCHK(c, launch_fx<T>(c->px, false, F, b.A, a, (const c2<T>*)twx, mkL(c, L, 0)));
  if (c->layered) {  // lateral transform only: [Kx][nz][Py] into the spectrum buffer
    LCHK(c, launch_fy<T>(c->py, true, b.A, b.S, a, (const c2<T>*)twy, mkL(c, L, 1)));
    return FR3D_OK;
  }
  LCHK(c, launch_fy<T>(c->py, true, b.A, b.B, a, (const c2<T>*)twy, mkL(c, L, 1)));
  LCHK(c, launch_fz<T>(c->pz, 0, b.B, b.S, a, (const c2<T>*)twz, mkL(c, L, 2)));
  return FR3D_OK;
}

LayArgs lay_args(fr3d_ctx* c) {
  LayArgs la{};
  la.M = c->g.nz;
  la.kxn = c->kxn;
  la.py = c->py;
  la.pyh = c->py / 2 + 1;
  la.kt = c->lay_kt;
  la.V = c->lay_V;
  la.lam = c->lay_lam;
  return la;
}

// slope: the seed of a secant search with a slope ratio, whose z pass also
// writes the partial sums of the full-box slope
template <typename T> fr3d_status inverse(fr3d_ctx* c, Lane& L, int mode, T* out, bool adj = false, bool slope = false) {
  const bool dbl = sizeof(T) == 8;
  void *twx, *twy, *twz;
  fr3d_status st;
  if ((st = get_twiddles(c, c->px, dbl, &twx)) || (st = get_twiddles(c, c->py, dbl, &twy)) ||
      (st = get_twiddles(c, c->pz, dbl, &twz)))
    return st;
  Bufs<T> b = bufs<T>(c, L);
  InvArgs a = inv_args(c, L, mode == 0);
  a.adj = adj ? 1 : 0;
  // the slope partials go to the z-pass bin partials, free between the
  // forward pass's features and the next data set
  if (slope && mode == 0 && !c->layered && c->filt == 0 && L.kmax == 0) {
    a.slope_part = (double2*)L.bins_part;
    if (!iz_slope_map<T>(c->pz, c->tile_sh[3], a) || (size_t)a.slope_n * (NT / 64) * 2 > c->bins_part_n * 64)
      return fail(c, FR3D_E_INVALID, "z pass of length %d: no slope partials", c->pz);
  }
  if (mode == 0 && L.kmax > 0) {
    // K-candidate step (runs only while the search is in that state)
    const size_t nA = (size_t)c->kxn * c->g.nz * c->g.ny, nB = (size_t)c->kxn * c->g.nz * c->py;
    InvArgs ak = a;
    ak.kmode = 1;
    ak.kmax = L.kmax;
    ak.w1_stride = (long long)nB;
    ak.w2_stride = (long long)nA;
    ak.norm_stride = (long long)c->norm_part_n;
    ak.norm_part = L.knorm;
    // candidates per z-pass workgroup: all K unless the grid would be small
    const long long tiles = (long long)c->kxn * std::max<long long>(1, (long long)c->py * c->pz / (c->esz == 8 ? 2048 : 4096));
    int kb = L.kmax;
    while (kb > 1 && tiles * ((L.kmax + kb - 1) / kb) < 2048) kb = (kb + 1) / 2;
    ak.kb = kb;
    c4<T>* W1k = (c4<T>*)L.kwork;
    c4<T>* W2k = W1k + (size_t)L.kmax * nB;
    const Launch none{L.stream, nullptr, nullptr, 0};
    Launch lz = none, ly = none, lx = none;
    lz.sh = 2;  // joint u/r tile: its loop over candidates keeps the fewest registers live
    ly.sh = c->tile_sh[4];
    lx.sh = c->tile_sh[5];
    if (c->layered) LCHK(c, launch_lay_filter<T>(0, b.S, W1k, lay_args(c), ak, lz));
    else LCHK(c, launch_iz<T>(c->pz, 0, b.S, W1k, ak, (const c2<T>*)twz, lz));
    LCHK(c, launch_iy<T>(c->py, W1k, W2k, ak, (const c2<T>*)twy, ly));
    LCHK(c, launch_ix<T>(c->px, 0, W2k, (T*)nullptr, ak, (const c2<T>*)twx, lx));
  }
  if (c->diag && mode == 0 && !c->layered) {
    InvArgs ad = a;
    ad.full_part = L.bins_part;  // free between the forward pass's features and the next data set
    constexpr int nb = 1024;
    hipLaunchKernelGGL(k_full_part<T>, dim3(nb), dim3(NT), 0, L.stream, (const c2<T>*)b.S, ad);
    hipLaunchKernelGGL(k_full_final, dim3(1), dim3(NT), 0, L.stream, ad, nb);
    LCHK(c, hipGetLastError());
  }
  if (c->layered) LCHK(c, launch_lay_filter<T>(mode, b.S, b.W1, lay_args(c), a, mkL(c, L, 3)));
  else LCHK(c, launch_iz<T>(c->pz, mode, b.S, b.W1, a, (const c2<T>*)twz, mkL(c, L, 3)));
  LCHK(c, launch_iy<T>(c->py, b.W1, b.W2, a, (const c2<T>*)twy, mkL(c, L, 4)));
  LCHK(c, launch_ix<T>(c->px, mode, b.W2, out, a, (const c2<T>*)twx, mkL(c, L, 5)));
  return FR3D_OK;
}

fr3d_status set_data_lane(fr3d_ctx* c, Lane& L, const void* F, double delta) {
  L.delta = delta;
  fr3d_status s = c->esz == 8 ? forward_data<double>(c, L, (const double*)F) : forward_data<float>(c, L, (const float*)F);
  if (s) return s;
  L.has_data = true;
  return FR3D_OK;
}

fr3d_status enqueue_eval(fr3d_ctx* c, Lane& L, bool slope = false) {
  return c->esz == 8 ? inverse<double>(c, L, 0, (double*)nullptr, false, slope)
                     : inverse<float>(c, L, 0, (float*)nullptr, false, slope);
}

// One evaluation of the lane's search (zeta goes where its control block
// says).  With graphs on, the launch sequence is captured once per lane
// (kernels only: every argument is fixed for the lane's geometry, the search
// state lives in the control block) and replayed.
fr3d_status eval_lane(fr3d_ctx* c, Lane& L) {
  if (L.slope_next) {  // the seed that forms the full-box slope: launched on its own
    L.slope_next = false;
    return enqueue_eval(c, L, true);
  }
  if (!c->graphs || c->timing) return enqueue_eval(c, L);
  if (!L.gexec || L.gkmax != L.kmax || std::memcmp(L.gsh, c->tile_sh, sizeof(L.gsh))) {
    if (L.gexec) (void)hipGraphExecDestroy(L.gexec);
    L.gexec = nullptr;
    if (!c->cap_stream) HIPCHK(c, hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    HIPCHK(c, hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    const hipStream_t keep = L.stream;
    L.stream = c->cap_stream;
    fr3d_status s = enqueue_eval(c, L);
    L.stream = keep;
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->cap_stream, &g);
    if (s) { if (g) (void)hipGraphDestroy(g); return s; }
    if (e != hipSuccess || !g) return fail(c, FR3D_E_DEVICE, "graph capture: %s", hipGetErrorString(e));
    const hipError_t e2 = hipGraphInstantiate(&L.gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) { L.gexec = nullptr; return fail(c, FR3D_E_DEVICE, "graph instantiate: %s", hipGetErrorString(e2)); }
    L.gkmax = L.kmax;
    std::memcpy(L.gsh, c->tile_sh, sizeof(L.gsh));
  }
  HIPCHK(c, hipGraphLaunch(L.gexec, L.stream));
  return FR3D_OK;
}

Ctrl ctrl_base(fr3d_ctx* c, Lane& L) {
  Ctrl v{};
  v.r2_full = -1.0;
  v.a_scale = c->g.alpha_relative ? c->smax : 1.0;
  v.delta = L.delta;
  v.tau = 1.0;
  v.h_op = 0.0;
  v.mu = 0.0;
  v.tol = 1e-3;
  v.acc_lo = 0.9;
  v.acc_hi = 1.1;
  v.lo = -8.0;
  v.hi = 0.0;
  v.walk = 0.25;
  v.max_steps = 40;
  v.active = 1;
  return v;
}

fr3d_status check_opts(fr3d_ctx* c, const fr3d_dp_opts* o, fr3d_dp_opts* d) {
  fr3d_dp_opts_default(d);
  if (o) *d = *o;
  if (!(d->log10_alpha_lo < d->log10_alpha_hi) || !std::isfinite(d->log10_alpha_lo) ||
      !std::isfinite(d->log10_alpha_hi) || d->max_steps < 0 || d->max_steps > 200 || !(d->tol >= 0) ||
      !(d->tau > 0) || !(d->h_op >= 0) || !(d->mu >= 0) || !(d->accept_lo <= d->accept_hi) ||
      !(d->seed_walk > 0) || !std::isfinite(d->seed_walk) || !(d->seed_slope >= 0) || !std::isfinite(d->seed_slope) || !std::isfinite(d->seed_slope_x) ||
      !(d->seed_snap_lo >= 0) || !std::isfinite(d->seed_snap_lo) || !(d->seed_slope_ratio >= 0) ||
      !std::isfinite(d->seed_slope_ratio))
    return fail(c, FR3D_E_INVALID, "bad search options");
  if (d->candidates != 0 && (d->candidates < 2 || d->candidates > KMAX || d->use_predictor || d->max_steps < 1))
    return fail(c, FR3D_E_INVALID, "candidates must be 2..%d, without use_predictor, with max_steps >= 1", KMAX);
  if (d->use_predictor && !c->has_pred) return fail(c, FR3D_E_STATE, "no predictor loaded");
  if (d->use_predictor && c->layered)
    return fail(c, FR3D_E_STATE, "the predictor's features come from the 3D spectrum (not with per-frequency systems)");
  return FR3D_OK;
}

fr3d_status ensure_kwork(fr3d_ctx* c, Lane& L, int K) {
  if (L.kcap >= K) return FR3D_OK;
  if (L.kpooled) return fail(c, FR3D_E_STATE, "lent K-candidate workspace holds fewer than %d candidates", K);
  dfree(L.kwork);
  dfree(L.knorm);
  L.kcap = 0;
  const size_t nA = (size_t)c->kxn * c->g.nz * c->g.ny, nB = (size_t)c->kxn * c->g.nz * c->py;
  HIPCHK(c, hipMalloc(&L.kwork, (size_t)K * (nA + nB) * 4 * c->esz));
  HIPCHK(c, hipMalloc(&L.knorm, (size_t)K * c->norm_part_n * sizeof(double2)));
  L.kcap = K;
  return FR3D_OK;
}

// Initial control block of a search with options d; with the predictor the
// first point is written on the device by the network's forward pass.
fr3d_status start_search(fr3d_ctx* c, Lane& L, const fr3d_dp_opts& d, void* zeta, int* max_evals) {
  Ctrl v = ctrl_base(c, L);
  v.out = zeta;
  v.lo = d.log10_alpha_lo;
  v.hi = d.log10_alpha_hi;
  v.max_steps = d.max_steps;
  v.tol = d.tol;
  v.acc_lo = d.accept_lo;
  v.acc_hi = d.accept_hi;
  v.tau = d.tau;
  v.h_op = d.h_op;
  v.mu = d.mu;
  v.walk = d.seed_walk;
  v.slope = d.seed_slope;
  v.slope_x = d.seed_slope_x;
  v.snap = d.seed_snap_lo;
  v.slope_ratio =
      (!d.candidates && d.use_predictor && d.seed_slope > 0 && c->filt == 0 && !c->layered) ? d.seed_slope_ratio : 0.0;
  L.slope_next = v.slope_ratio > 0;  // the next evaluation is the seed
  v.slope_full = -1.0;
  v.state = ST_HI;
  v.t = v.hi;
  v.alpha_abs = std::pow(10.0, v.hi) * v.a_scale;
  L.kmax = 0;
  if (d.candidates) {
    fr3d_status s = ensure_kwork(c, L, d.candidates);
    if (s) return s;
    L.kmax = d.candidates;
    v.state = ST_KARY;
    v.kmax = d.candidates;
    v.steps = 0;
    const size_t nB = (size_t)c->kxn * c->g.nz * c->py;
    v.kw1 = L.kwork;
    v.kw2 = (char*)L.kwork + (size_t)d.candidates * nB * 4 * c->esz;
    v.knorm = L.knorm;
  }
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(1), 0, L.stream, L.ctrl, v);
  LCHK(c, hipGetLastError());
  if (d.candidates) {
    *max_evals = d.max_steps;  // each evaluation call: one K-candidate step, then the answer once found
  } else if (d.use_predictor) {
    LCHK(c, mlp_forward(c->pred_p, c->pred_norm, L.feat, 1, nullptr, nullptr, L.ctrl, L.stream,
                        c->has_cal ? c->pred_cal : nullptr));
    if (d.seed_slope > 0) {
      *max_evals = 1 + d.max_steps + 1;  // seed + secant steps + final re-evaluation
    } else {
      // seed + doubling walk across the range + regula falsi + final re-evaluation
      int walk = 0;
      for (double w = d.seed_walk, span = 0; span < d.log10_alpha_hi - d.log10_alpha_lo; w *= 2) { span += w; ++walk; }
      *max_evals = 1 + walk + d.max_steps + 1;
    }
  } else {
    *max_evals = 2 + d.max_steps + 1;
  }
  return FR3D_OK;
}

fr3d_status fixed_search(fr3d_ctx* c, Lane& L, double alpha, void* zeta) {
  L.kmax = 0;
  L.slope_next = false;
  Ctrl v = ctrl_base(c, L);
  v.out = zeta;
  v.state = ST_FIXED;
  v.t = std::log10(alpha);
  v.alpha_abs = alpha * v.a_scale;
  hipLaunchKernelGGL(k_ctrl_init, dim3(1), dim3(1), 0, L.stream, L.ctrl, v);
  LCHK(c, hipGetLastError());
  return FR3D_OK;
}

fr3d_status post_ctrl(fr3d_ctx* c, Lane& L) {
  HIPCHK(c, hipMemcpyAsync(L.ctrl_host, L.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, L.stream));
  HIPCHK(c, hipEventRecord(L.ev, L.stream));
  return FR3D_OK;
}

void fill_report(const Ctrl& h, fr3d_report* r) {
  r->alpha = std::pow(10.0, h.t);
  r->residual = std::sqrt(h.r2);
  r->zeta_norm = std::sqrt(h.z2);
  r->delta = h.delta;
  r->target = h.target;
  r->n_evals = h.n_evals;
  r->flags = h.flags;
  r->n_clamped = -1;
  r->residual_full_box = h.r2_full >= 0 ? std::sqrt(h.r2_full) : -1.0;
}

int env_int(const char* name, int dflt) {
  const char* s = std::getenv(name);
  return s ? std::atoi(s) : dflt;
}

// Single search on lane 0, chunks of evaluations between host reads.
fr3d_status run_search(fr3d_ctx* c, int max_evals, fr3d_report* rep) {
  Lane& L = c->lanes[0];
  const int chunk = std::max(1, env_int("FR3D_EVAL_CHUNK", 4));
  int launched = 0;
  fr3d_status s;
  for (;;) {
    const int k = std::min(chunk, max_evals - launched);
    for (int i = 0; i < k; ++i)
      if ((s = eval_lane(c, L))) return s;
    launched += k;
    if ((s = post_ctrl(c, L))) return s;
    HIPCHK(c, hipEventSynchronize(L.ev));
    if (!L.ctrl_host->active || launched >= max_evals) break;
  }
  if (c->timing) tcollect(c, L, L.ctrl_host->n_evals);
  if (L.ctrl_host->active) return fail(c, FR3D_E_DEVICE, "alpha search did not finish in %d evaluations", max_evals);
  if (rep) fill_report(*L.ctrl_host, rep);
  return FR3D_OK;
}

// The whole search on lane 0 with no host read: max_evals evaluations (those
// after the search has ended return at once), then the report on the device.
fr3d_status enqueue_search(fr3d_ctx* c, int max_evals, fr3d_report* rep_dev) {
  Lane& L = c->lanes[0];
  fr3d_status s;
  for (int i = 0; i < max_evals; ++i)
    if ((s = enqueue_eval(c, L, i == 0 && L.slope_next))) return s;
  L.slope_next = false;
  hipLaunchKernelGGL(k_report, dim3(1), dim3(1), 0, L.stream, (const Ctrl*)L.ctrl, rep_dev);
  LCHK(c, hipGetLastError());
  return FR3D_OK;
}

bool need(fr3d_ctx* c, bool kernel, bool data) {
  if (kernel && !c->has_kernel) { fail(c, FR3D_E_STATE, "no kernel loaded"); return false; }
  if (data && !c->lanes[0].has_data) { fail(c, FR3D_E_STATE, "no data set"); return false; }
  return true;
}

long long ncells(fr3d_ctx* c) { return (long long)c->g.nx * c->g.ny * c->g.nz; }

// Workgroups of a recovery over n cells (grid-stride beyond), one clamp-count partial each.
constexpr int RECOVER_MAX_BLOCKS = 2048;
unsigned recover_blocks(long long n) { return (unsigned)std::min<long long>((n + NT - 1) / NT, RECOVER_MAX_BLOCKS); }

fr3d_status launch_recover(fr3d_ctx* c, Lane& L, const void* zeta, const void* V0, double c0, void* cout,
                           bool count) {
  const long long n = ncells(c);
  double* part = (double*)L.norm_part;  // >= 2 nz ny doubles
  const double ic2 = 1.0 / (c0 * c0), fl = 1e-6 / (c0 * c0);
  const unsigned nb = recover_blocks(n);
  if (c->esz == 8)
    hipLaunchKernelGGL(k_recover<double>, dim3(nb), dim3(NT), 0, L.stream, (const double*)zeta, (const double*)V0,
                       ic2, fl, (double*)cout, n, part);
  else
    hipLaunchKernelGGL(k_recover<float>, dim3(nb), dim3(NT), 0, L.stream, (const float*)zeta, (const float*)V0, ic2,
                       fl, (float*)cout, n, part);
  LCHK(c, hipGetLastError());
  if (count) {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(NT), 0, L.stream, (const double*)part, (int)nb, 1, 1, L.scal);
    LCHK(c, hipGetLastError());
    HIPCHK(c, hipMemcpyAsync(L.scal_host, L.scal, sizeof(double), hipMemcpyDeviceToHost, L.stream));
  }
  return FR3D_OK;
}

fr3d_status ensure_lanes(fr3d_ctx* c) {
  const int want = std::max(1, c->nlanes_wanted);
  while ((int)c->lanes.size() < want) {
    hipStream_t s;
    HIPCHK(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    c->lanes.emplace_back();
    Lane& L = c->lanes.back();
    fr3d_status st = init_lane(c, L, s, true);
    if (st) return st;
    if (c->has_kernel && (st = alloc_lane_geometry(c, L))) return st;
  }
  return FR3D_OK;
}

fr3d_status pred_ensure_work(fr3d_ctx* c, int B) {
  if (B <= c->pred_cap && c->pred_work) return FR3D_OK;
  dfree(c->pred_work);
  const int cap = std::max(B, 256);
  HIPCHK(c, hipMalloc(&c->pred_work, mlp_work_bytes(cap)));
  c->pred_cap = cap;
  return FR3D_OK;
}

fr3d_status pred_alloc(fr3d_ctx* c) {
  if (c->pred_p) return FR3D_OK;
  HIPCHK(c, hipMalloc(&c->pred_p, MLP_NP * sizeof(float)));
  HIPCHK(c, hipMalloc(&c->pred_m, MLP_NP * sizeof(float)));
  HIPCHK(c, hipMalloc(&c->pred_v, MLP_NP * sizeof(float)));
  HIPCHK(c, hipMalloc(&c->pred_g, MLP_NP * sizeof(float)));
  HIPCHK(c, hipMalloc(&c->pred_norm, MLP_NNORM * sizeof(float)));
  HIPCHK(c, hipMalloc(&c->pred_loss, 4 * sizeof(float)));
  return FR3D_OK;
}

uint64_t fnv1a(const void* data, size_t n, uint64_t h = 1469598103934665603ull) {
  const unsigned char* p = (const unsigned char*)data;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
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
  o->seed_walk = 0.25;
  o->seed_slope = 0.0;
  o->seed_slope_x = 0.0;
  o->seed_snap_lo = 0.0;
  o->seed_slope_ratio = 0.0;
  o->candidates = 0;
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
  c->lanes.emplace_back();
  if (init_lane(c, c->lanes[0], (hipStream_t)stream, false) != FR3D_OK || hipDeviceSynchronize() != hipSuccess) {
    fr3d_destroy(c);
    return FR3D_E_NOMEM;
  }
  *out = c;
  return FR3D_OK;
}

fr3d_status fr3d_destroy(fr3d_ctx* c) {
  if (!c) return FR3D_E_INVALID;
  (void)hipSetDevice(c->device);
  for (auto& L : c->lanes) (void)hipStreamSynchronize(L.stream);
  free_geometry(c);
  for (auto& L : c->lanes) {
    for (int p = 0; p < 6; ++p)
      for (auto& e : L.tev[p]) c->ev_pool.push_back(e);
    free_lane(L);
  }
  for (auto& e : c->ev_pool) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  for (auto& p : c->pool_kw) dfree(p);
  for (auto& p : c->pool_kn) dfree(p);
  dfree(c->cg_buf);
  dfree(c->pf_part);
  dfree(c->cg_part);
  dfree(c->cg_dev);
  hfree(c->cg_host);
  dfree(c->pred_p);
  dfree(c->pred_m);
  dfree(c->pred_v);
  dfree(c->pred_g);
  dfree(c->pred_norm);
  dfree(c->pred_cal);
  dfree(c->pred_loss);
  dfree(c->pred_work);
  delete c;
  return FR3D_OK;
}

fr3d_status fr3d_set_stream(fr3d_ctx* c, void* stream) {
  if (!c) return FR3D_E_INVALID;
  c->lanes[0].stream = (hipStream_t)stream;
  return FR3D_OK;
}

fr3d_status fr3d_set_lanes(fr3d_ctx* c, int32_t lanes) {
  if (!c) return FR3D_E_INVALID;
  if (lanes < 1 || lanes > 64) return fail(c, FR3D_E_INVALID, "lanes must be in [1, 64]");
  c->nlanes_wanted = lanes;
  return ensure_lanes(c);
}

// Per-workgroup largest deviation of the samples from evenness in x and y
// (part[b]) and largest magnitude (part[nb + b]).
__global__ void k_even_dev(const double* __restrict__ k, int px, int py, int pz, double* part) {
  __shared__ double rd[NT], rm[NT];
  double dev = 0.0, mag = 0.0;
  const long long n = (long long)px * py * pz;
  for (long long e = (long long)blockIdx.x * NT + threadIdx.x; e < n; e += (long long)gridDim.x * NT) {
    const int x = (int)(e % px), y = (int)((e / px) % py);
    const long long z = e / ((long long)px * py);
    const double v = k[e];
    const double vx = k[(z * py + y) * px + (px - x) % px];
    const double vy = k[(z * py + (py - y) % py) * px + x];
    dev = fmax(dev, fmax(fabs(v - vx), fabs(v - vy)));
    mag = fmax(mag, fabs(v));
  }
  rd[threadIdx.x] = dev;
  rm[threadIdx.x] = mag;
  __syncthreads();
  for (int s = NT / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      rd[threadIdx.x] = fmax(rd[threadIdx.x], rd[threadIdx.x + s]);
      rm[threadIdx.x] = fmax(rm[threadIdx.x], rm[threadIdx.x + s]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = rd[0];
    part[gridDim.x + blockIdx.x] = rm[0];
  }
}

fr3d_status load_kernel_impl(fr3d_ctx* c, const fr3d_geom* g, const double* ksrc);

fr3d_status fr3d_load_kernel(fr3d_ctx* c, const fr3d_geom* g) { return load_kernel_impl(c, g, nullptr); }

fr3d_status fr3d_load_kernel_samples(fr3d_ctx* c, const fr3d_geom* g, const double* k_dev) {
  if (!c) return FR3D_E_INVALID;
  if (!k_dev) return fail(c, FR3D_E_INVALID, "k_dev is null");
  return load_kernel_impl(c, g, k_dev);
}

fr3d_status load_kernel_impl(fr3d_ctx* c, const fr3d_geom* g, const double* ksrc) {
  if (!c) return FR3D_E_INVALID;
  if (!g) return fail(c, FR3D_E_INVALID, "geom is null");
  if (g->nx < 2 || g->ny < 2 || g->nz < 2) return fail(c, FR3D_E_INVALID, "grid extents must be >= 2");
  if (!supported_length(2 * g->nx) || !supported_length(2 * g->ny) || !supported_length(2 * g->nz))
    return fail(c, FR3D_E_INVALID, "2n per axis must be one of the compiled lengths (2^a 3^b, <= 512)");
  if (!(g->h > 0) || !std::isfinite(g->h)) return fail(c, FR3D_E_INVALID, "h must be finite and > 0");
  if (!std::isfinite(g->hz)) return fail(c, FR3D_E_INVALID, "hz must be finite");
  if (g->kind != 0 && g->kind != 1) return fail(c, FR3D_E_INVALID, "kind must be 0 or 1");
  if (g->precision != 32 && g->precision != 64) return fail(c, FR3D_E_INVALID, "precision must be 32 or 64");
  if (!std::isfinite(g->D)) return fail(c, FR3D_E_INVALID, "D must be finite");
  if (g->alpha_relative != 0 && g->alpha_relative != 1) return fail(c, FR3D_E_INVALID, "alpha_relative must be 0 or 1");
  const double D = g->D > 0 ? g->D : (double)gap_default(g->nz, g->q);
  if (D < g->nz) return fail(c, FR3D_E_INVALID, "D must be >= nz (R and Y disjoint)");
  HIPCHK(c, hipSetDevice(c->device));
  for (auto& L : c->lanes) HIPCHK(c, L.stream ? hipStreamSynchronize(L.stream) : hipDeviceSynchronize());
  free_geometry(c);
  c->g = *g;
  c->D = D;
  c->hz = g->hz > 0 ? g->hz : g->h;
  c->px = 2 * g->nx; c->py = 2 * g->ny; c->pz = 2 * g->nz;
  c->kxn = c->px / 2 + 1;
  c->esz = g->precision == 64 ? 8 : 4;
  const size_t kxn = c->kxn;
  const size_t nS = kxn * spec_plane(c->pz, c->py, spec_lg(c->esz, c->pz, c->py));  // column-granule layout
  const size_t nA = kxn * g->nz * g->ny, nB = kxn * g->nz * c->py;
  c->spec_bytes = nS * 2 * c->esz;
  c->work_bytes = (nA + nB) * 4 * c->esz;  // W1 + W2 (pairs) cover A + B
  c->bins_part_n = (size_t)kxn * c->py + 64;  // >= workgroups of the z pass (tile pairs, padded grid)
  c->norm_part_n = (size_t)g->nz * g->ny;  // >= workgroups of the x pass
  const size_t noct = kxn * (c->pz / 2 + 1) * (c->py / 2 + 1);
  fr3d_status st;
  if (ksrc) {
    // the octant form needs a real table even in x and y
    Lane& Lv = c->lanes[0];
    constexpr int nb = 512;
    double* part = nullptr;
    HIPCHK(c, hipMalloc(&part, 2 * nb * sizeof(double)));
    hipLaunchKernelGGL(k_even_dev, dim3(nb), dim3(NT), 0, Lv.stream, ksrc, c->px, c->py, c->pz, part);
    hipLaunchKernelGGL(k_max_parts, dim3(1), dim3(NT), 0, Lv.stream, (const double*)part, nb, Lv.scal);
    hipLaunchKernelGGL(k_max_parts, dim3(1), dim3(NT), 0, Lv.stream, (const double*)(part + nb), nb, Lv.scal + 1);
    hipError_t ev = hipGetLastError();
    if (ev == hipSuccess) ev = hipMemcpyAsync(Lv.scal_host, Lv.scal, 2 * sizeof(double), hipMemcpyDeviceToHost, Lv.stream);
    if (ev == hipSuccess) ev = hipStreamSynchronize(Lv.stream);
    (void)hipFree(part);
    if (ev != hipSuccess) return fail(c, FR3D_E_DEVICE, "kernel samples check: %s", hipGetErrorString(ev));
    const double dev = Lv.scal_host[0], mag = Lv.scal_host[1];
    if (!std::isfinite(dev) || !std::isfinite(mag) || !(mag > 0)) {
      c->has_kernel = false;
      return fail(c, FR3D_E_INVALID, "kernel samples must be finite and not all zero");
    }
    if (dev > 1e-12 * mag) {
      c->has_kernel = false;
      return fail(c, FR3D_E_INVALID, "kernel samples must be even in x and y (relative deviation %.3g)", dev / mag);
    }
  }
  HIPCHK(c, hipMalloc(&c->oct, noct * sizeof(double2)));
  for (auto& L : c->lanes)
    if ((st = alloc_lane_geometry(c, L))) return st;
  Lane& L0 = c->lanes[0];
  // kernel spectrum in FP64 through full (unpruned) passes; temporaries freed after
  double2 *Ak = nullptr, *Bk = nullptr;
  HIPCHK(c, hipMalloc(&Ak, nS * sizeof(double2)));
  hipError_t e2 = hipMalloc(&Bk, nS * sizeof(double2));
  if (e2 != hipSuccess) { (void)hipFree(Ak); return fail(c, FR3D_E_NOMEM, "kernel spectrum workspace: %s", hipGetErrorString(e2)); }
  void *twx, *twy, *twz;
  if ((st = get_twiddles(c, c->px, true, &twx)) || (st = get_twiddles(c, c->py, true, &twy)) ||
      (st = get_twiddles(c, c->pz, true, &twz))) {
    (void)hipFree(Ak); (void)hipFree(Bk);
    return st;
  }
  FwdArgs a = fwd_args(c, L0, true);
  a.ksrc = ksrc;
  const Launch Lk{L0.stream, nullptr, nullptr, 0};
  hipError_t le = launch_fx<double>(c->px, true, nullptr, Ak, a, (const double2*)twx, Lk);
  if (le == hipSuccess) le = launch_fy<double>(c->py, false, Ak, Bk, a, (const double2*)twy, Lk);
  if (le == hipSuccess) le = launch_fz<double>(c->pz, 1, Bk, c->oct, a, (const double2*)twz, Lk);
  const unsigned nb = (unsigned)std::min<long long>(((long long)noct + NT - 1) / NT, 1024);
  if (le == hipSuccess) {
    hipLaunchKernelGGL(k_smax_part, dim3(nb), dim3(NT), 0, L0.stream, c->oct, (long long)noct, (double*)Ak);
    le = hipGetLastError();
  }
  if (le == hipSuccess) {
    hipLaunchKernelGGL(k_max_parts, dim3(1), dim3(NT), 0, L0.stream, (const double*)Ak, (int)nb, L0.scal);
    le = hipGetLastError();
  }
  if (le == hipSuccess) le = hipMemcpyAsync(L0.scal_host, L0.scal, sizeof(double), hipMemcpyDeviceToHost, L0.stream);
  if (le == hipSuccess) le = hipStreamSynchronize(L0.stream);
  (void)hipFree(Ak);
  (void)hipFree(Bk);
  if (le != hipSuccess) return fail(c, FR3D_E_DEVICE, "kernel spectrum: %s", hipGetErrorString(le));
  c->smax = L0.scal_host[0];
  if (!(c->smax > 0) || !std::isfinite(c->smax)) return fail(c, FR3D_E_DEVICE, "kernel spectrum has no energy");
  {
    // levels of the kernel spectrum for the predictor features: thresholds
    // s_max 10^((j - 64)/4), j = 1..63
    LevelThr thr;
    for (int j = 1; j < 64; ++j) thr.t[j - 1] = c->smax * std::pow(10.0, (j - 64) / 4.0);
    HIPCHK(c, hipMalloc(&c->level, (size_t)kxn * (c->py / 2 + 1) * c->pz));
    const unsigned nr = (unsigned)std::min<long long>(((long long)noct + NT - 1) / NT, 4096);
    hipLaunchKernelGGL(k_level_table, dim3(nr), dim3(NT), 0, L0.stream, (const double2*)c->oct, c->kxn,
                       c->pz / 2 + 1, c->py / 2 + 1, c->pz, thr, c->level);
    LCHK(c, hipGetLastError());
  }
  if (c->esz == 4) {
    HIPCHK(c, hipMalloc(&c->oct32, noct * sizeof(float2)));
    const unsigned nr = (unsigned)std::min<long long>(((long long)noct + NT - 1) / NT, 4096);
    hipLaunchKernelGGL(k_round_octant, dim3(nr), dim3(NT), 0, L0.stream, (const double2*)c->oct, (long long)noct, c->oct32);
    LCHK(c, hipGetLastError());
  }
  const bool dbl = c->esz == 8;
  if ((st = get_twiddles(c, c->px, dbl, &twx)) || (st = get_twiddles(c, c->py, dbl, &twy)) ||
      (st = get_twiddles(c, c->pz, dbl, &twz)))
    return st;
  c->has_kernel = true;
  return FR3D_OK;
}

fr3d_status fr3d_load_layered(fr3d_ctx* c, const fr3d_geom* g) {
  if (!c) return FR3D_E_INVALID;
  if (!g) return fail(c, FR3D_E_INVALID, "geom is null");
  if (g->nx < 2 || g->ny < 2 || g->nz < 1) return fail(c, FR3D_E_INVALID, "need nx, ny >= 2 and nz >= 1");
  if (g->nz > LAY_MMAX) return fail(c, FR3D_E_INVALID, "nz must be <= %d for the per-frequency systems", LAY_MMAX);
  if (!supported_length(2 * g->nx) || !supported_length(2 * g->ny))
    return fail(c, FR3D_E_INVALID, "2n per lateral axis must be one of the compiled lengths (2^a 3^b, <= 512)");
  if (!(g->h > 0) || !std::isfinite(g->h)) return fail(c, FR3D_E_INVALID, "h must be finite and > 0");
  if (!std::isfinite(g->hz)) return fail(c, FR3D_E_INVALID, "hz must be finite");
  if (g->kind != 0 && g->kind != 1) return fail(c, FR3D_E_INVALID, "kind must be 0 or 1");
  if (g->precision != 32 && g->precision != 64) return fail(c, FR3D_E_INVALID, "precision must be 32 or 64");
  if (!std::isfinite(g->D)) return fail(c, FR3D_E_INVALID, "D must be finite");
  if (g->alpha_relative != 0 && g->alpha_relative != 1) return fail(c, FR3D_E_INVALID, "alpha_relative must be 0 or 1");
  const double D = g->D > 0 ? g->D : (double)gap_default(g->nz, g->q);
  if (D < g->nz) return fail(c, FR3D_E_INVALID, "D must be >= nz (R and Y disjoint)");
  HIPCHK(c, hipSetDevice(c->device));
  for (auto& L : c->lanes) HIPCHK(c, L.stream ? hipStreamSynchronize(L.stream) : hipDeviceSynchronize());
  free_geometry(c);
  c->g = *g;
  c->D = D;
  c->hz = g->hz > 0 ? g->hz : g->h;
  c->px = 2 * g->nx; c->py = 2 * g->ny; c->pz = 2 * g->nz;
  c->kxn = c->px / 2 + 1;
  c->esz = g->precision == 64 ? 8 : 4;
  const size_t kxn = c->kxn, M = g->nz, Lz = 2 * M - 1, pyh = c->py / 2 + 1, nf = kxn * pyh;
  const size_t nA = kxn * g->nz * g->ny, nB = kxn * g->nz * c->py;
  c->spec_bytes = nB * 2 * c->esz;         // lateral spectrum [Kx][nz][Py]
  c->work_bytes = (nA + nB) * 4 * c->esz;  // W1 + W2 (pairs) cover A
  c->bins_part_n = (size_t)kxn * c->py;
  c->norm_part_n = (size_t)g->nz * g->ny;
  HIPCHK(c, hipMalloc(&c->lay_kt, nf * Lz * sizeof(double)));
  HIPCHK(c, hipMalloc(&c->lay_V, nf * M * M * sizeof(double)));
  HIPCHK(c, hipMalloc(&c->lay_lam, nf * M * sizeof(double)));
  c->layered = true;
  fr3d_status st;
  for (auto& L : c->lanes)
    if ((st = alloc_lane_geometry(c, L))) return st;
  Lane& L0 = c->lanes[0];
  // lateral transform of the kernel at the 2 nz - 1 z offsets (FP64), then the SVDs
  const size_t nk = kxn * Lz * c->py;
  double2 *Ak = nullptr, *Bk = nullptr;
  HIPCHK(c, hipMalloc(&Ak, nk * sizeof(double2)));
  hipError_t e2 = hipMalloc(&Bk, nk * sizeof(double2));
  if (e2 != hipSuccess) { (void)hipFree(Ak); return fail(c, FR3D_E_NOMEM, "kernel transform workspace: %s", hipGetErrorString(e2)); }
  void *twx, *twy;
  if ((st = get_twiddles(c, c->px, true, &twx)) || (st = get_twiddles(c, c->py, true, &twy))) {
    (void)hipFree(Ak); (void)hipFree(Bk);
    return st;
  }
  FwdArgs a = fwd_args(c, L0, true);
  a.nz_in = (int)Lz;
  a.zlin = 1;
  const Launch Lk{L0.stream, nullptr, nullptr, 0};
  LayArgs la = lay_args(c);
  hipError_t le = launch_fx<double>(c->px, true, nullptr, Ak, a, (const double2*)twx, Lk);
  if (le == hipSuccess) le = launch_fy<double>(c->py, false, Ak, Bk, a, (const double2*)twy, Lk);
  if (le == hipSuccess) le = launch_lay_svd(Bk, la, c->lay_kt, c->lay_V, c->lay_lam, L0.stream);
  if (le == hipSuccess) le = launch_lay_max(c->lay_lam, (long long)(nf * M), (double*)Ak, L0.scal, L0.stream);
  if (le == hipSuccess) le = hipMemcpyAsync(L0.scal_host, L0.scal, sizeof(double), hipMemcpyDeviceToHost, L0.stream);
  if (le == hipSuccess) le = hipStreamSynchronize(L0.stream);
  (void)hipFree(Ak);
  (void)hipFree(Bk);
  if (le != hipSuccess) return fail(c, FR3D_E_DEVICE, "per-frequency systems: %s", hipGetErrorString(le));
  c->smax = L0.scal_host[0];
  if (!(c->smax > 0) || !std::isfinite(c->smax)) return fail(c, FR3D_E_DEVICE, "kernel has no energy");
  const bool dbl = c->esz == 8;
  if ((st = get_twiddles(c, c->px, dbl, &twx)) || (st = get_twiddles(c, c->py, dbl, &twy))) return st;
  c->has_kernel = true;
  return FR3D_OK;
}

fr3d_status fr3d_set_data(fr3d_ctx* c, const void* F, double delta) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!F) return fail(c, FR3D_E_INVALID, "F is null");
  if (!(delta >= 0) || !std::isfinite(delta)) return fail(c, FR3D_E_INVALID, "delta must be finite and >= 0");
  return set_data_lane(c, c->lanes[0], F, delta);
}

fr3d_status fr3d_solve_alpha(fr3d_ctx* c, double alpha, void* zeta, fr3d_report* rep) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, true)) return FR3D_E_STATE;
  if (!zeta) return fail(c, FR3D_E_INVALID, "zeta is null");
  if (!(alpha > 0) || !std::isfinite(alpha)) return fail(c, FR3D_E_INVALID, "alpha must be finite and > 0");
  fr3d_status s = fixed_search(c, c->lanes[0], alpha, zeta);
  if (s) return s;
  return run_search(c, 1, rep);
}

fr3d_status fr3d_solve_discrepancy(fr3d_ctx* c, const fr3d_dp_opts* o, void* zeta, fr3d_report* rep) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, true)) return FR3D_E_STATE;
  if (!zeta) return fail(c, FR3D_E_INVALID, "zeta is null");
  fr3d_dp_opts d;
  fr3d_status s = check_opts(c, o, &d);
  if (s) return s;
  int max_evals = 0;
  if ((s = start_search(c, c->lanes[0], d, zeta, &max_evals))) return s;
  return run_search(c, max_evals, rep);
}

fr3d_status fr3d_solve_alpha_dev(fr3d_ctx* c, double alpha, void* zeta, fr3d_report* rep_dev) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, true)) return FR3D_E_STATE;
  if (!zeta || !rep_dev) return fail(c, FR3D_E_INVALID, "zeta or rep_dev is null");
  if (!(alpha > 0) || !std::isfinite(alpha)) return fail(c, FR3D_E_INVALID, "alpha must be finite and > 0");
  if (c->timing) return fail(c, FR3D_E_STATE, "timing is on (host-side events); turn it off for _dev solves");
  fr3d_status s = fixed_search(c, c->lanes[0], alpha, zeta);
  if (s) return s;
  return enqueue_search(c, 1, rep_dev);
}

fr3d_status fr3d_solve_discrepancy_dev(fr3d_ctx* c, const fr3d_dp_opts* o, void* zeta, fr3d_report* rep_dev) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, true)) return FR3D_E_STATE;
  if (!zeta || !rep_dev) return fail(c, FR3D_E_INVALID, "zeta or rep_dev is null");
  if (c->timing) return fail(c, FR3D_E_STATE, "timing is on (host-side events); turn it off for _dev solves");
  fr3d_dp_opts d;
  fr3d_status s = check_opts(c, o, &d);
  if (s) return s;
  int max_evals = 0;
  if ((s = start_search(c, c->lanes[0], d, zeta, &max_evals))) return s;
  return enqueue_search(c, max_evals, rep_dev);
}

}  // extern "C"

namespace {

// Scheduler over slots (a slot = a context and one of its lanes).  Item i
// runs set_data, the search and (optionally) recovery on one slot whose
// context is ctx_of[i]; each slot advances one evaluation at a time, and the
// host polls the slots' completion events and enqueues the next step of
// whichever slot is ready, so the slots' work overlaps on the device and no
// evaluation is launched after its search has finished.
struct Slot {
  fr3d_ctx* c;
  int lane;
};

struct Items {
  int n;
  fr3d_ctx* const* ctx_of;  // per item, or null: every item on ctx0
  fr3d_ctx* ctx0;
  const void* const* F;
  const double* deltas;
  void* const* zetas;
  const void* const* V0;  // per item (null: no recovery)
  double c0;
  void* const* c_out;
  float* feat_out;
  fr3d_report* reps;
};

// Pooled K-candidate workspaces of a group solve: an item starts only when a
// slot is free and holds it until its lane is idle again.
struct KLend {
  fr3d_ctx* owner;
  int K;
  std::vector<int> free_slots;
};

void lend(KLend* kl, Lane& L, int slot) {
  L.own_kwork = L.kwork;
  L.own_knorm = L.knorm;
  L.own_kcap = L.kcap;
  L.kwork = kl->owner->pool_kw[slot];
  L.knorm = kl->owner->pool_kn[slot];
  L.kcap = kl->K;
  L.kpooled = true;
}

void give_back(Lane& L) {
  L.kwork = L.own_kwork;
  L.knorm = L.own_knorm;
  L.kcap = L.own_kcap;
  L.own_kwork = nullptr;
  L.own_knorm = nullptr;
  L.kpooled = false;
}

fr3d_status run_schedule(std::vector<Slot>& slots, const Items& it, const fr3d_dp_opts& d, KLend* kl = nullptr) {
  const int ns = (int)slots.size();
  enum { IDLE, SEARCH, RECOVER };
  std::vector<int> item(ns, -1), state(ns, IDLE), launched(ns, 0), limit(ns, 0), held(ns, -1);
  std::vector<char> started(it.n, 0);
  int done = 0, scan = 0;
  fr3d_status s = FR3D_OK;
  fr3d_ctx* bad = nullptr;
  auto ctx_of = [&](int i) { return it.ctx_of ? it.ctx_of[i] : it.ctx0; };
  while (done < it.n && s == FR3D_OK) {
    bool progressed = false;
    for (int l = 0; l < ns && s == FR3D_OK; ++l) {
      fr3d_ctx* c = slots[l].c;
      Lane& L = c->lanes[slots[l].lane];
      if (state[l] == IDLE) {
        int i = -1;
        for (int k = scan; k < it.n; ++k)
          if (!started[k] && ctx_of(k) == c) { i = k; break; }
        if (i < 0) continue;
        if (kl) {  // the item needs a pooled workspace
          if (kl->free_slots.empty()) continue;
          held[l] = kl->free_slots.back();
          kl->free_slots.pop_back();
          lend(kl, L, held[l]);
        }
        started[i] = 1;
        while (scan < it.n && started[scan]) ++scan;
        item[l] = i;
        bad = c;
        if ((s = set_data_lane(c, L, it.F[i], it.deltas[i]))) break;
        if (it.feat_out && hipMemcpyAsync(it.feat_out + (size_t)i * 65, L.feat, 65 * sizeof(float),
                                          hipMemcpyDeviceToDevice, L.stream) != hipSuccess) {
          s = fail(c, FR3D_E_DEVICE, "feature copy");
          break;
        }
        if ((s = start_search(c, L, d, it.zetas[i], &limit[l]))) break;
        if ((s = eval_lane(c, L))) break;
        launched[l] = 1;
        if ((s = post_ctrl(c, L))) break;
        state[l] = SEARCH;
        progressed = true;
        continue;
      }
      const hipError_t q = hipEventQuery(L.ev);
      if (q == hipErrorNotReady) continue;
      bad = c;
      if (q != hipSuccess) { s = fail(c, FR3D_E_DEVICE, "lane %d: %s", slots[l].lane, hipGetErrorString(q)); break; }
      progressed = true;
      const int i = item[l];
      if (state[l] == SEARCH) {
        if (L.ctrl_host->active && launched[l] < limit[l]) {
          if ((s = eval_lane(c, L))) break;
          launched[l] += 1;
          if ((s = post_ctrl(c, L))) break;
          continue;
        }
        if (L.ctrl_host->active) { s = fail(c, FR3D_E_DEVICE, "search of item %d did not finish", i); break; }
        fill_report(*L.ctrl_host, &it.reps[i]);
        if (c->timing) tcollect(c, L, L.ctrl_host->n_evals);
        if (it.c_out) {
          if ((s = launch_recover(c, L, it.zetas[i], it.V0[i], it.c0, it.c_out[i], true))) break;
          if (hipEventRecord(L.ev, L.stream) != hipSuccess) { s = fail(c, FR3D_E_DEVICE, "event record"); break; }
          state[l] = RECOVER;
          continue;
        }
      } else {
        it.reps[i].n_clamped = (int64_t)L.scal_host[0];
      }
      state[l] = IDLE;
      if (held[l] >= 0) {
        give_back(L);
        kl->free_slots.push_back(held[l]);
        held[l] = -1;
      }
      done += 1;
    }
    if (!progressed && s == FR3D_OK) std::this_thread::yield();
  }
  if (kl)  // after an error: lanes still holding a slot wait for their work, then return it
    for (int l = 0; l < ns; ++l)
      if (held[l] >= 0) {
        Lane& L = slots[l].c->lanes[slots[l].lane];
        (void)hipStreamSynchronize(L.stream);
        give_back(L);
        kl->free_slots.push_back(held[l]);
        held[l] = -1;
      }
  if (s != FR3D_OK && bad && it.ctx0 && bad != it.ctx0) it.ctx0->err = bad->err;
  return s;
}

// Orders every lane in use of c after (begin) or before (end) c's lane 0.
fr3d_status fence_lanes(fr3d_ctx* c, int nl, bool begin) {
  hipEvent_t e;
  HIPCHK(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
  if (begin) {
    HIPCHK(c, hipEventRecord(e, c->lanes[0].stream));
    for (int l = 1; l < nl; ++l) HIPCHK(c, hipStreamWaitEvent(c->lanes[l].stream, e, 0));
  } else {
    for (int l = 1; l < nl; ++l) {
      HIPCHK(c, hipEventRecord(e, c->lanes[l].stream));
      HIPCHK(c, hipStreamWaitEvent(c->lanes[0].stream, e, 0));
    }
  }
  (void)hipEventDestroy(e);
  return FR3D_OK;
}

fr3d_status check_item(fr3d_ctx* c, int i, const void* F, double delta, void* zeta, bool rec, const void* V0,
                       void* cout) {
  if (!F || !zeta || (rec && (!cout || !V0))) return fail(c, FR3D_E_INVALID, "null array in batch item %d", i);
  if (!(delta >= 0) || !std::isfinite(delta)) return fail(c, FR3D_E_INVALID, "bad delta in batch item %d", i);
  return FR3D_OK;
}

}  // namespace

extern "C" {

fr3d_status fr3d_solve_batch(fr3d_ctx* c, int32_t n, const void* const* F, const double* deltas, void* const* zetas,
                             const fr3d_dp_opts* o, const void* V0, double c0, void* const* c_out,
                             float* feat_out, fr3d_report* reps) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (n < 0 || (n > 0 && (!F || !deltas || !zetas || !reps))) return fail(c, FR3D_E_INVALID, "null batch arrays");
  if (c_out && (!V0 || !(c0 > 0) || !std::isfinite(c0))) return fail(c, FR3D_E_INVALID, "recovery needs V0 and c0 > 0");
  if (feat_out && c->layered) return fail(c, FR3D_E_STATE, "no features with per-frequency systems");
  fr3d_status s;
  for (int i = 0; i < n; ++i)
    if ((s = check_item(c, i, F[i], deltas[i], zetas[i], c_out != nullptr, V0, c_out ? c_out[i] : nullptr))) return s;
  fr3d_dp_opts d;
  if ((s = check_opts(c, o, &d))) return s;
  if ((s = ensure_lanes(c))) return s;
  const int nl = std::max(1, std::min((int)c->lanes.size(), c->nlanes_wanted));
  std::vector<Slot> slots;
  for (int l = 0; l < nl; ++l) slots.push_back({c, l});
  std::vector<const void*> v0s(c_out ? n : 0, V0);
  Items it{n, nullptr, c, F, deltas, zetas, c_out ? v0s.data() : nullptr, c0, c_out, feat_out, reps};
  if ((s = fence_lanes(c, nl, true))) return s;
  s = run_schedule(slots, it, d);
  fence_lanes(c, nl, false);
  if (s != FR3D_OK)
    for (auto& L : c->lanes) (void)hipStreamSynchronize(L.stream);
  return s;
}

// Items of different geometries (grid sizes, kernels) in one scheduler: item
// i runs on ctxs[i]; every lane in use of every distinct context is a slot.
fr3d_status fr3d_solve_group(int32_t n, fr3d_ctx* const* ctxs, const void* const* F, const double* deltas,
                             void* const* zetas, const fr3d_dp_opts* o, const void* const* V0s, double c0,
                             void* const* c_out, fr3d_report* reps) {
  if (n < 0 || (n > 0 && (!ctxs || !ctxs[0]))) return FR3D_E_INVALID;
  if (n == 0) return FR3D_OK;
  fr3d_ctx* c0x = ctxs[0];
  if (!F || !deltas || !zetas || !reps) return fail(c0x, FR3D_E_INVALID, "null batch arrays");
  if (c_out && (!V0s || !(c0 > 0) || !std::isfinite(c0))) return fail(c0x, FR3D_E_INVALID, "recovery needs V0 and c0 > 0");
  std::vector<fr3d_ctx*> distinct;
  fr3d_status s;
  for (int i = 0; i < n; ++i) {
    fr3d_ctx* c = ctxs[i];
    if (!c) return fail(c0x, FR3D_E_INVALID, "null context in item %d", i);
    if (!need(c, true, false)) { c0x->err = c->err; return FR3D_E_STATE; }
    if ((s = check_item(c0x, i, F[i], deltas[i], zetas[i], c_out != nullptr, c_out ? V0s[i] : nullptr,
                        c_out ? c_out[i] : nullptr)))
      return s;
    if (std::find(distinct.begin(), distinct.end(), c) == distinct.end()) distinct.push_back(c);
  }
  fr3d_dp_opts d;
  for (fr3d_ctx* c : distinct)
    if ((s = check_opts(c, o, &d))) { c0x->err = c->err; return s; }
  std::vector<Slot> slots;
  std::vector<int> nls;
  for (fr3d_ctx* c : distinct) {
    if ((s = ensure_lanes(c))) { c0x->err = c->err; return s; }
    const int nl = std::max(1, std::min((int)c->lanes.size(), c->nlanes_wanted));
    nls.push_back(nl);
    if ((s = fence_lanes(c, nl, true))) { c0x->err = c->err; return s; }
    for (int l = 0; l < nl; ++l) slots.push_back({c, l});
  }
  Items it{n, ctxs, c0x, F, deltas, zetas, V0s, c0, c_out, nullptr, reps};
  KLend kl{c0x, d.candidates, {}};
  if (d.candidates) {
    // pooled K-candidate workspaces (slots on ctxs[0], reused by later calls)
    size_t kwb = 0, knb = 0;
    for (fr3d_ctx* c : distinct) {
      const size_t nA = (size_t)c->kxn * c->g.nz * c->g.ny, nB = (size_t)c->kxn * c->g.nz * c->py;
      kwb = std::max(kwb, (size_t)d.candidates * (nA + nB) * 4 * c->esz);
      knb = std::max(knb, (size_t)d.candidates * c->norm_part_n * sizeof(double2));
    }
    const int want = std::max(1, std::min((int)slots.size(), env_int("FR3D_GROUP_KSLOTS", 8)));
    if (c0x->pool_kw_bytes < kwb || c0x->pool_kn_bytes < knb) {
      for (fr3d_ctx* c : distinct)
        for (auto& L : c->lanes) (void)hipStreamSynchronize(L.stream);
      for (auto& p : c0x->pool_kw) dfree(p);
      for (auto& p : c0x->pool_kn) dfree(p);
      c0x->pool_kw.clear();
      c0x->pool_kn.clear();
      c0x->pool_kw_bytes = kwb;
      c0x->pool_kn_bytes = knb;
    }
    while ((int)c0x->pool_kw.size() < want) {
      void* w = nullptr;
      double2* k = nullptr;
      HIPCHK(c0x, hipMalloc(&w, c0x->pool_kw_bytes));
      c0x->pool_kw.push_back(w);
      HIPCHK(c0x, hipMalloc(&k, c0x->pool_kn_bytes));
      c0x->pool_kn.push_back(k);
    }
    for (int k = 0; k < want; ++k) kl.free_slots.push_back(want - 1 - k);
  }
  s = run_schedule(slots, it, d, d.candidates ? &kl : nullptr);
  for (size_t k = 0; k < distinct.size(); ++k) fence_lanes(distinct[k], nls[k], false);
  if (s != FR3D_OK)
    for (fr3d_ctx* c : distinct)
      for (auto& L : c->lanes) (void)hipStreamSynchronize(L.stream);
  return s;
}

fr3d_status fr3d_recover_c(fr3d_ctx* c, const void* zeta, const void* V0, double c0, void* cout, int64_t* ncl) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!zeta || !V0 || !cout) return fail(c, FR3D_E_INVALID, "null array");
  if (!(c0 > 0) || !std::isfinite(c0)) return fail(c, FR3D_E_INVALID, "c0 must be finite and > 0");
  Lane& L = c->lanes[0];
  fr3d_status s = launch_recover(c, L, zeta, V0, c0, cout, ncl != nullptr);
  if (s) return s;
  if (ncl) {
    HIPCHK(c, hipStreamSynchronize(L.stream));
    *ncl = (int64_t)L.scal_host[0];
  }
  return FR3D_OK;
}

}  // extern "C"

// ------------------------------------------------------------ no-allocation recovery
// Scratch of fr3d_recover_c_noalloc: the per-workgroup clamp-count partials
// (16 KiB).  Each device holds its own copy for the life of the process;
// host code reaches it only through the address hipGetSymbolAddress returns
// for the current device (the array's name in host code is not a device
// address).
static __device__ __align__(256) double scratch[RECOVER_MAX_BLOCKS];

namespace {

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex noalloc_mu;
double* noalloc_ptr[NOALLOC_MAX_DEVICES] = {};

// The current device's scratch address, looked up once per device with that
// device current; null if the device is not a usable gfx950 or the lookup fails.
double* noalloc_scratch() {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return nullptr;
  std::lock_guard<std::mutex> lk(noalloc_mu);
  if (noalloc_ptr[dev]) return noalloc_ptr[dev];
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, dev) != hipSuccess || std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
    return nullptr;
  void* ptr = nullptr;
  if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return nullptr;
  noalloc_ptr[dev] = (double*)ptr;
  return noalloc_ptr[dev];
}

}  // namespace

extern "C" {

fr3d_status fr3d_recover_c_noalloc(int32_t precision, int64_t n, const void* zeta, const void* V0, double c0,
                                   void* cout, int64_t* ncl_dev, void* stream) {
  if (precision != 32 && precision != 64) return FR3D_E_INVALID;
  if (n < 0 || n > FR3D_NOALLOC_MAX_CELLS) return FR3D_E_INVALID;
  if (n > 0 && (!zeta || !V0 || !cout)) return FR3D_E_INVALID;
  if (!(c0 > 0) || !std::isfinite(c0)) return FR3D_E_INVALID;
  double* part = noalloc_scratch();
  if (!part) return FR3D_E_DEVICE;
  const hipStream_t st = (hipStream_t)stream;
  const unsigned nb = recover_blocks(n);
  const double ic2 = 1.0 / (c0 * c0), fl = 1e-6 / (c0 * c0);
  if (nb > 0) {
    if (precision == 64)
      hipLaunchKernelGGL(k_recover<double>, dim3(nb), dim3(NT), 0, st, (const double*)zeta, (const double*)V0, ic2,
                         fl, (double*)cout, (long long)n, part);
    else
      hipLaunchKernelGGL(k_recover<float>, dim3(nb), dim3(NT), 0, st, (const float*)zeta, (const float*)V0, ic2, fl,
                         (float*)cout, (long long)n, part);
    if (hipGetLastError() != hipSuccess) return FR3D_E_DEVICE;
  }
  if (ncl_dev) {
    hipLaunchKernelGGL(k_clamp_count, dim3(1), dim3(NT), 0, st, (const double*)part, (int)nb, ncl_dev);
    if (hipGetLastError() != hipSuccess) return FR3D_E_DEVICE;
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
      s.z[5 * k + l] = hz[k] * c->hz;
    }
  const long long n = ncells(c);
  Lane& L = c->lanes[0];
  dim3 grid((unsigned)std::min<long long>((n + 255) / 256, 4096));
  if (c->esz == 8)
    hipLaunchKernelGGL(k_v0<double>, grid, dim3(256), 0, L.stream, (double*)V0, c->g.nx, c->g.ny, c->g.nz, h, c->hz, A0, s);
  else
    hipLaunchKernelGGL(k_v0<float>, grid, dim3(256), 0, L.stream, (float*)V0, c->g.nx, c->g.ny, c->g.nz, h, c->hz, A0, s);
  LCHK(c, hipGetLastError());
  return FR3D_OK;
}

}  // extern "C"

namespace {

constexpr int CG_PARTS = 1024;

fr3d_status cg_alloc(fr3d_ctx* c) {
  const size_t bytes = 4 * (size_t)ncells(c) * c->esz;
  if (c->cg_cap < bytes) {
    dfree(c->cg_buf);
    c->cg_cap = 0;
    HIPCHK(c, hipMalloc(&c->cg_buf, bytes));
    c->cg_cap = bytes;
  }
  if (!c->cg_part) HIPCHK(c, hipMalloc(&c->cg_part, CG_PARTS * sizeof(double)));
  if (!c->cg_dev) HIPCHK(c, hipMalloc(&c->cg_dev, 8 * sizeof(double)));
  if (!c->cg_host) HIPCHK(c, hipHostMalloc(&c->cg_host, 8 * sizeof(double), hipHostMallocDefault));
  return FR3D_OK;
}

// out = A in (adj = false: R -> Y) or A^T in (adj = true: Y -> R) through
// lane 0's buffers (its data spectrum is overwritten).
template <typename T> fr3d_status apply_lin(fr3d_ctx* c, const T* in, T* out, bool adj) {
  Lane& L = c->lanes[0];
  fr3d_status s;
  if ((s = forward_data<T>(c, L, in))) return s;
  L.has_data = false;
  return inverse<T>(c, L, 1, out, adj);
}

// Sum of the per-block partials into cg[slot] (one workgroup, fixed order).
fr3d_status cg_sum(fr3d_ctx* c, hipStream_t st, int nb, int slot) {
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(NT), 0, st, (const double*)c->cg_part, nb, 1, 1, c->cg_dev + slot);
  LCHK(c, hipGetLastError());
  return FR3D_OK;
}

// CG on (A^T A + a I) x = A^T F from x = 0 until ||r|| <= tol ||A^T F||
// (checked every 16 steps) or max_iter steps; then ||A x - F||_Y and ||x||_R.
template <typename T>
fr3d_status cg_solve(fr3d_ctx* c, const T* F, double a, T* x, int max_iter, double tol, int* iters, bool* conv,
                     double* rnorm, double* xnorm) {
  fr3d_status s;
  if ((s = cg_alloc(c))) return s;
  const long long n = ncells(c);
  T* r = (T*)c->cg_buf;
  T* p = r + n;
  T* q = p + n;
  T* t = q + n;
  hipStream_t st = c->lanes[0].stream;
  const int nb = (int)std::min<long long>((n + NT - 1) / NT, CG_PARTS);
  if ((s = apply_lin<T>(c, F, r, true))) return s;  // r = b = A^T F
  hipLaunchKernelGGL(k_fill0<T>, dim3(nb), dim3(NT), 0, st, x, n);
  HIPCHK(c, hipMemcpyAsync(p, r, n * sizeof(T), hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL(k_dot_part<T>, dim3(nb), dim3(NT), 0, st, (const T*)r, (const T*)r, n, c->cg_part);
  LCHK(c, hipGetLastError());
  if ((s = cg_sum(c, st, nb, 0))) return s;
  HIPCHK(c, hipMemcpyAsync(c->cg_dev + 3, c->cg_dev, sizeof(double), hipMemcpyDeviceToDevice, st));
  int it = 0;
  bool done = false;
  for (;;) {
    if (it % 16 == 0 || it >= max_iter) {
      HIPCHK(c, hipMemcpyAsync(c->cg_host, c->cg_dev, 4 * sizeof(double), hipMemcpyDeviceToHost, st));
      HIPCHK(c, hipStreamSynchronize(st));
      const double rr = c->cg_host[0], bb = c->cg_host[3];
      if (!std::isfinite(rr)) return fail(c, FR3D_E_DEVICE, "CG residual is not finite");
      if (bb == 0.0 || rr <= tol * tol * bb) { done = true; break; }
      if (it >= max_iter) break;
    }
    if ((s = apply_lin<T>(c, p, t, false))) return s;  // t = A p
    if ((s = apply_lin<T>(c, t, q, true))) return s;   // q = A^T A p
    hipLaunchKernelGGL(k_cg_q<T>, dim3(nb), dim3(NT), 0, st, q, (const T*)p, a, n, c->cg_part);
    LCHK(c, hipGetLastError());
    if ((s = cg_sum(c, st, nb, 1))) return s;
    hipLaunchKernelGGL(k_cg_step<T>, dim3(nb), dim3(NT), 0, st, x, r, (const T*)p, (const T*)q, n,
                       (const double*)c->cg_dev, c->cg_part);
    LCHK(c, hipGetLastError());
    if ((s = cg_sum(c, st, nb, 2))) return s;
    hipLaunchKernelGGL(k_cg_dir<T>, dim3(nb), dim3(NT), 0, st, p, (const T*)r, n, (const double*)c->cg_dev);
    hipLaunchKernelGGL(k_cg_roll, dim3(1), dim3(1), 0, st, c->cg_dev);
    LCHK(c, hipGetLastError());
    ++it;
  }
  // residual on Y and norm on R of the estimate
  if ((s = apply_lin<T>(c, x, t, false))) return s;
  hipLaunchKernelGGL(k_sub_sq<T>, dim3(nb), dim3(NT), 0, st, t, F, n, c->cg_part);
  LCHK(c, hipGetLastError());
  if ((s = cg_sum(c, st, nb, 5))) return s;
  hipLaunchKernelGGL(k_dot_part<T>, dim3(nb), dim3(NT), 0, st, (const T*)x, (const T*)x, n, c->cg_part);
  LCHK(c, hipGetLastError());
  if ((s = cg_sum(c, st, nb, 4))) return s;
  HIPCHK(c, hipMemcpyAsync(c->cg_host, c->cg_dev, 8 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  *iters = it;
  *conv = done;
  *rnorm = std::sqrt(c->cg_host[5]);
  *xnorm = std::sqrt(c->cg_host[4]);
  return FR3D_OK;
}

fr3d_status exact_eval(fr3d_ctx* c, const void* F, double alpha_abs, void* x, int max_iter, double tol, int* iters,
                       bool* conv, double* rn, double* xn) {
  return c->esz == 8 ? cg_solve<double>(c, (const double*)F, alpha_abs, (double*)x, max_iter, tol, iters, conv, rn, xn)
                     : cg_solve<float>(c, (const float*)F, alpha_abs, (float*)x, max_iter, tol, iters, conv, rn, xn);
}

fr3d_status check_exact(fr3d_ctx* c, const void* F, void* zeta, int max_iter, double tol) {
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!F || !zeta) return fail(c, FR3D_E_INVALID, "null array");
  if (max_iter < 1) return fail(c, FR3D_E_INVALID, "max_iter must be >= 1");
  if (!(tol > 0) || !std::isfinite(tol)) return fail(c, FR3D_E_INVALID, "tol must be finite and > 0");
  return FR3D_OK;
}

}  // namespace

extern "C" {

fr3d_status fr3d_solve_per_frequency(fr3d_ctx* c, const fr3d_dp_opts* o, void* zeta, double* alpha_dev,
                                     int32_t* flags_dev, fr3d_report* rep) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, true)) return FR3D_E_STATE;
  if (!c->layered) return fail(c, FR3D_E_STATE, "per-frequency alphas need the per-frequency systems (fr3d_load_layered)");
  if (!zeta) return fail(c, FR3D_E_INVALID, "zeta is null");
  fr3d_dp_opts d;
  fr3d_status s = check_opts(c, o, &d);
  if (s) return s;
  if (d.use_predictor || d.candidates || d.h_op != 0 || d.mu != 0)
    return fail(c, FR3D_E_INVALID, "the per-frequency search is the plain rule (no predictor, candidates, h_op or mu)");
  Lane& L = c->lanes[0];
  const size_t nf = (size_t)c->kxn * (c->py / 2 + 1);
  if (c->pf_cap < nf) {
    dfree(c->pf_part);
    c->pf_cap = 0;
    HIPCHK(c, hipMalloc(&c->pf_part, nf * 5 * sizeof(double)));
    c->pf_cap = nf;
  }
  if ((s = fixed_search(c, L, 1.0, zeta))) return s;  // one spatial evaluation: norms and zeta on R
  PfArgs pf{};
  pf.target = d.tau * L.delta;
  pf.a_scale = c->g.alpha_relative ? c->smax : 1.0;
  pf.lo = d.log10_alpha_lo;
  pf.hi = d.log10_alpha_hi;
  pf.tol = d.tol;
  pf.max_steps = d.max_steps;
  pf.alpha_out = alpha_dev;
  pf.flags_out = (int*)flags_dev;
  pf.part = c->pf_part;
  const bool dbl = c->esz == 8;
  void *twx, *twy;
  if ((s = get_twiddles(c, c->px, dbl, &twx)) || (s = get_twiddles(c, c->py, dbl, &twy))) return s;
  InvArgs a = inv_args(c, L, true);
  const Launch none{L.stream, nullptr, nullptr, 0};
  Launch ly = none, lx = none;
  ly.sh = c->tile_sh[4];
  lx.sh = c->tile_sh[5];
  if (dbl) {
    Bufs<double> b = bufs<double>(c, L);
    LCHK(c, launch_lay_pf<double>(b.S, b.W1, lay_args(c), a, pf, none));
    LCHK(c, launch_iy<double>(c->py, b.W1, b.W2, a, (const c2<double>*)twy, ly));
    LCHK(c, launch_ix<double>(c->px, 0, b.W2, (double*)nullptr, a, (const c2<double>*)twx, lx));
  } else {
    Bufs<float> b = bufs<float>(c, L);
    LCHK(c, launch_lay_pf<float>(b.S, b.W1, lay_args(c), a, pf, none));
    LCHK(c, launch_iy<float>(c->py, b.W1, b.W2, a, (const c2<float>*)twy, ly));
    LCHK(c, launch_ix<float>(c->px, 0, b.W2, (float*)nullptr, a, (const c2<float>*)twx, lx));
  }
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(NT), 0, L.stream, (const double*)c->pf_part, (int)nf, 5, 5, L.scal);
  LCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(L.scal_host, L.scal, 5 * sizeof(double), hipMemcpyDeviceToHost, L.stream));
  if ((s = post_ctrl(c, L))) return s;
  HIPCHK(c, hipEventSynchronize(L.ev));
  if (L.ctrl_host->active) return fail(c, FR3D_E_DEVICE, "per-frequency evaluation did not finish");
  if (rep) {
    fill_report(*L.ctrl_host, rep);
    const double* sc = L.scal_host;
    rep->alpha = std::pow(10.0, sc[0] / sc[1]);
    rep->delta = L.delta;
    rep->target = pf.target;
    rep->n_evals = 1;
    rep->flags = (sc[2] > 0 ? FR3D_NOROOT_HIGH : 0) | (sc[3] > 0 ? FR3D_NOROOT_LOW : 0) | (sc[4] > 0 ? FR3D_MAXITER : 0);
  }
  return FR3D_OK;
}

fr3d_status fr3d_solve_exact(fr3d_ctx* c, const void* F, double alpha, void* zeta, int32_t max_iter, double tol,
                             fr3d_report* rep) {
  if (!c) return FR3D_E_INVALID;
  fr3d_status s;
  if ((s = check_exact(c, F, zeta, max_iter, tol))) return s;
  if (!(alpha > 0) || !std::isfinite(alpha)) return fail(c, FR3D_E_INVALID, "alpha must be finite and > 0");
  const double a_scale = c->g.alpha_relative ? c->smax : 1.0;
  int iters = 0;
  bool conv = false;
  double rn = 0, xn = 0;
  if ((s = exact_eval(c, F, alpha * a_scale, zeta, max_iter, tol, &iters, &conv, &rn, &xn))) return s;
  if (rep) {
    *rep = fr3d_report{};
    rep->alpha = alpha;
    rep->residual = rn;
    rep->zeta_norm = xn;
    rep->n_evals = iters;
    rep->flags = conv ? 0 : FR3D_CG_LIMIT;
    rep->n_clamped = -1;
    rep->residual_full_box = -1.0;
  }
  return FR3D_OK;
}

fr3d_status fr3d_solve_exact_discrepancy(fr3d_ctx* c, const void* F, double delta, const fr3d_dp_opts* o, void* zeta,
                                         int32_t max_iter, double tol, fr3d_report* rep) {
  if (!c) return FR3D_E_INVALID;
  fr3d_status s;
  if ((s = check_exact(c, F, zeta, max_iter, tol))) return s;
  if (!(delta >= 0) || !std::isfinite(delta)) return fail(c, FR3D_E_INVALID, "delta must be >= 0");
  fr3d_dp_opts d;
  if ((s = check_opts(c, o, &d))) return s;
  if (d.use_predictor || d.candidates) return fail(c, FR3D_E_INVALID, "the exact-operator search is the plain rule");
  const double a_scale = c->g.alpha_relative ? c->smax : 1.0;
  // the plain rule (bisection in log10 alpha), as on the device for the other forms
  int n_evals = 0, flags = 0;
  double r = 0, zn = 0, tgt = 0, last_t = 0;
  auto ev = [&](double t, double* rho, double* ratio) -> fr3d_status {
    int iters = 0;
    bool conv = false;
    fr3d_status e = exact_eval(c, F, std::pow(10.0, t) * a_scale, zeta, max_iter, tol, &iters, &conv, &r, &zn);
    if (e) return e;
    if (!conv) flags |= FR3D_CG_LIMIT;
    ++n_evals;
    last_t = t;
    const double g = d.tau * delta + d.h_op * zn;
    const double t2 = g * g + d.mu * d.mu;
    tgt = std::sqrt(t2);
    *rho = r * r - t2;
    *ratio = t2 > 0 ? r / tgt : INFINITY;
    return FR3D_OK;
  };
  double rho = 0, ratio = 0, t = d.log10_alpha_hi;
  auto finish = [&](double tt, int fl) {
    if (rep) {
      *rep = fr3d_report{};
      rep->alpha = std::pow(10.0, tt);
      rep->residual = r;
      rep->zeta_norm = zn;
      rep->delta = delta;
      rep->target = tgt;
      rep->n_evals = n_evals;
      rep->flags = flags | fl;
      rep->n_clamped = -1;
      rep->residual_full_box = -1.0;
    }
    return FR3D_OK;
  };
  if ((s = ev(d.log10_alpha_hi, &rho, &ratio))) return s;
  if (std::fabs(ratio - 1.0) <= d.tol) return finish(d.log10_alpha_hi, 0);
  if (rho < 0) return finish(d.log10_alpha_hi, FR3D_NOROOT_HIGH);
  if ((s = ev(d.log10_alpha_lo, &rho, &ratio))) return s;
  if (std::fabs(ratio - 1.0) <= d.tol) return finish(d.log10_alpha_lo, 0);
  if (rho > 0) return finish(d.log10_alpha_lo, FR3D_NOROOT_LOW);
  double a = d.log10_alpha_lo, b = d.log10_alpha_hi;
  for (int k = 0; k < d.max_steps; ++k) {
    t = 0.5 * (a + b);
    if ((s = ev(t, &rho, &ratio))) return s;
    if (std::fabs(ratio - 1.0) <= d.tol) return finish(t, 0);
    if (rho < 0) a = t;
    else b = t;
  }
  if (last_t != b && (s = ev(b, &rho, &ratio))) return s;
  return finish(b, FR3D_MAXITER);
}

fr3d_status fr3d_apply_operator(fr3d_ctx* c, const void* zeta, void* F) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!zeta || !F) return fail(c, FR3D_E_INVALID, "null array");
  Lane& L = c->lanes[0];
  fr3d_status s;
  if (c->esz == 8) {
    if ((s = forward_data<double>(c, L, (const double*)zeta))) return s;
    s = inverse<double>(c, L, 1, (double*)F);
  } else {
    if ((s = forward_data<float>(c, L, (const float*)zeta))) return s;
    s = inverse<float>(c, L, 1, (float*)F);
  }
  L.has_data = false;  // the spectrum buffer now holds zeta's transform
  return s;
}

fr3d_status fr3d_add_noise(fr3d_ctx* c, void* F, const void* e, double delta_rel, double* delta) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!F || !e) return fail(c, FR3D_E_INVALID, "null array");
  if (!(delta_rel >= 0) || !std::isfinite(delta_rel)) return fail(c, FR3D_E_INVALID, "delta_rel must be >= 0");
  Lane& L = c->lanes[0];
  const long long n = ncells(c);
  const unsigned nb = (unsigned)std::min<long long>((n + NT - 1) / NT, 1024);
  double* nrm = L.scal + 2;
  double* part = (double*)L.norm_part;
  if (c->esz == 8)
    hipLaunchKernelGGL(k_norms2<double>, dim3(nb), dim3(NT), 0, L.stream, (const double*)F, (const double*)e, n, part);
  else
    hipLaunchKernelGGL(k_norms2<float>, dim3(nb), dim3(NT), 0, L.stream, (const float*)F, (const float*)e, n, part);
  LCHK(c, hipGetLastError());
  hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(NT), 0, L.stream, (const double*)part, (int)nb, 2, 2, nrm);
  LCHK(c, hipGetLastError());
  dim3 grid((unsigned)std::min<long long>((n + 255) / 256, 4096));
  if (c->esz == 8)
    hipLaunchKernelGGL(k_add_noise<double>, grid, dim3(256), 0, L.stream, (double*)F, (const double*)e, n, delta_rel, nrm);
  else
    hipLaunchKernelGGL(k_add_noise<float>, grid, dim3(256), 0, L.stream, (float*)F, (const float*)e, n, delta_rel, nrm);
  LCHK(c, hipGetLastError());
  HIPCHK(c, hipMemcpyAsync(L.scal_host, nrm, 2 * sizeof(double), hipMemcpyDeviceToHost, L.stream));
  HIPCHK(c, hipStreamSynchronize(L.stream));
  if (delta) *delta = delta_rel * std::sqrt(L.scal_host[0]);
  return FR3D_OK;
}

fr3d_status fr3d_get_octant(fr3d_ctx* c, void* out, int64_t bytes) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (c->layered) return fail(c, FR3D_E_STATE, "no 3D kernel spectrum with per-frequency systems");
  const size_t n = (size_t)c->kxn * (c->pz / 2 + 1) * (c->py / 2 + 1) * sizeof(double2);
  if (!out || bytes < (int64_t)n) return fail(c, FR3D_E_INVALID, "need %zu bytes", n);
  HIPCHK(c, hipMemcpyAsync(out, c->oct, n, hipMemcpyDeviceToDevice, c->lanes[0].stream));
  return FR3D_OK;
}

fr3d_status fr3d_get_singular_values(fr3d_ctx* c, double* out, int64_t bytes) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  if (!c->layered) return fail(c, FR3D_E_STATE, "singular values belong to the per-frequency systems (fr3d_load_layered)");
  const size_t n = (size_t)c->kxn * (c->py / 2 + 1) * c->g.nz * sizeof(double);
  if (!out || bytes < (int64_t)n) return fail(c, FR3D_E_INVALID, "need %zu bytes", n);
  LCHK(c, launch_lay_sv(lay_args(c), out, c->lanes[0].stream));
  return FR3D_OK;
}

fr3d_status fr3d_get_data_spectrum(fr3d_ctx* c, void* out, int64_t bytes) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  // the layered form's lateral spectrum as stored; the 3D spectrum in the
  // standard layout [Kx][Pz][Py] (stored in column granules)
  const size_t nb = c->layered ? c->spec_bytes : (size_t)c->kxn * c->pz * c->py * 2 * c->esz;
  if (!out || bytes < (int64_t)nb) return fail(c, FR3D_E_INVALID, "need %zu bytes", nb);
  Lane& L0 = c->lanes[0];
  if (c->layered) {
    HIPCHK(c, hipMemcpyAsync(out, L0.spec, nb, hipMemcpyDeviceToDevice, L0.stream));
  } else {
    const long long n = (long long)c->kxn * c->pz * c->py;
    const unsigned g = (unsigned)std::min<long long>((n + NT - 1) / NT, 8192);
    if (c->esz == 8)
      hipLaunchKernelGGL(k_spec_untile<double>, dim3(g), dim3(NT), 0, L0.stream, (const double2*)L0.spec,
                         (double2*)out, c->kxn, c->pz, c->py);
    else
      hipLaunchKernelGGL(k_spec_untile<float>, dim3(g), dim3(NT), 0, L0.stream, (const float2*)L0.spec,
                         (float2*)out, c->kxn, c->pz, c->py);
    LCHK(c, hipGetLastError());
  }
  return FR3D_OK;
}

fr3d_status fr3d_get_features(fr3d_ctx* c, float* feat, double* energy) {
  if (!c) return FR3D_E_INVALID;
  if (!need(c, true, true)) return FR3D_E_STATE;
  if (c->layered) return fail(c, FR3D_E_STATE, "features come from the 3D spectrum (not with per-frequency systems)");
  Lane& L = c->lanes[0];
  if (feat) HIPCHK(c, hipMemcpyAsync(feat, L.feat, 65 * sizeof(float), hipMemcpyDeviceToDevice, L.stream));
  if (energy) HIPCHK(c, hipMemcpyAsync(energy, L.energy, 64 * sizeof(double), hipMemcpyDeviceToDevice, L.stream));
  return FR3D_OK;
}

fr3d_status fr3d_get_smax(fr3d_ctx* c, double* smax) {
  if (!c || !smax) return FR3D_E_INVALID;
  if (!need(c, true, false)) return FR3D_E_STATE;
  *smax = c->smax;
  return FR3D_OK;
}

fr3d_status fr3d_set_tile(fr3d_ctx* c, int32_t pass, int32_t shift) {
  if (!c) return FR3D_E_INVALID;
  if (pass < 0 || pass > 5) return fail(c, FR3D_E_INVALID, "pass must be in [0, 5]");
  const int maxsh = (pass == 0 || pass == 1 || pass == 3 || pass == 4) ? 2 : 1;
  if (shift < 0 || (shift & 3) > maxsh || (shift >> 2) > 2)
    return fail(c, FR3D_E_INVALID, "tile shift of pass %d must be in [0, %d] plus 4 v with a plan variant v in [0, 2]",
                pass, maxsh);
  c->tile_sh[pass] = shift;
  return FR3D_OK;
}

fr3d_status fr3d_set_filter(fr3d_ctx* c, int32_t kind, int32_t order) {
  if (!c) return FR3D_E_INVALID;
  if (kind < 0 || kind > 2) return fail(c, FR3D_E_INVALID, "filter kind must be 0, 1 or 2");
  if (kind == 1 && (order < 1 || order > 64)) return fail(c, FR3D_E_INVALID, "iterated Tikhonov order must be in [1, 64]");
  for (auto& L : c->lanes) (void)hipStreamSynchronize(L.stream);
  c->filt = kind;
  c->forder = kind == 1 ? order : 1;
  // captured evaluations hold the old filter in their arguments
  for (auto& L : c->lanes) {
    if (L.gexec) (void)hipGraphExecDestroy(L.gexec);
    L.gexec = nullptr;
  }
  return FR3D_OK;
}

fr3d_status fr3d_set_diagnostics(fr3d_ctx* c, int32_t enable) {
  if (!c) return FR3D_E_INVALID;
  for (auto& L : c->lanes) (void)hipStreamSynchronize(L.stream);
  c->diag = enable != 0;
  // captured evaluations hold the old launch sequence
  for (auto& L : c->lanes) {
    if (L.gexec) (void)hipGraphExecDestroy(L.gexec);
    L.gexec = nullptr;
  }
  return FR3D_OK;
}

fr3d_status fr3d_set_graphs(fr3d_ctx* c, int32_t enable) {
  if (!c) return FR3D_E_INVALID;
  c->graphs = enable != 0;
  return FR3D_OK;
}

fr3d_status fr3d_set_timing(fr3d_ctx* c, int32_t enable) {
  if (!c) return FR3D_E_INVALID;
  for (auto& L : c->lanes) {
    (void)hipStreamSynchronize(L.stream);
    tcollect(c, L);
  }
  c->timing = enable != 0;
  return FR3D_OK;
}

fr3d_status fr3d_get_timing(fr3d_ctx* c, int32_t pass, double* total_ms, int64_t* launches) {
  if (!c || pass < 0 || pass > 5) return FR3D_E_INVALID;
  for (auto& L : c->lanes) {
    (void)hipStreamSynchronize(L.stream);
    tcollect(c, L);
  }
  if (total_ms) *total_ms = c->acc_ms[pass];
  if (launches) *launches = c->cnt[pass];
  c->acc_ms[pass] = 0;
  c->cnt[pass] = 0;
  return FR3D_OK;
}

// ------------------------------------------------------------ predictor
fr3d_status fr3d_predictor_set(fr3d_ctx* c, const float* params, int64_t n_params, const float* norm) {
  if (!c) return FR3D_E_INVALID;
  if (!params || !norm || n_params != MLP_NP) return fail(c, FR3D_E_INVALID, "need %d parameters and norm[%d]", MLP_NP, MLP_NNORM);
  for (int i = 0; i < MLP_IN; ++i)
    if (!(norm[MLP_IN + i] > 0) || !std::isfinite(norm[MLP_IN + i]))
      return fail(c, FR3D_E_INVALID, "feature deviations must be finite and > 0");
  if (!(norm[2 * MLP_IN + 1] > 0) || !std::isfinite(norm[2 * MLP_IN + 1]))
    return fail(c, FR3D_E_INVALID, "target deviation must be finite and > 0");
  fr3d_status s = pred_alloc(c);
  if (s) return s;
  hipStream_t st = c->lanes[0].stream;
  HIPCHK(c, hipMemcpyAsync(c->pred_p, params, MLP_NP * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->pred_norm, norm, MLP_NNORM * sizeof(float), hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemsetAsync(c->pred_m, 0, MLP_NP * sizeof(float), st));
  HIPCHK(c, hipMemsetAsync(c->pred_v, 0, MLP_NP * sizeof(float), st));
  HIPCHK(c, hipStreamSynchronize(st));
  c->pred_step = 0;
  c->has_pred = true;
  c->has_cal = false;  // a calibration belongs to the network it was fitted for
  return FR3D_OK;
}

fr3d_status fr3d_predictor_set_calibration(fr3d_ctx* c, const double* coef, int64_t n) {
  if (!c) return FR3D_E_INVALID;
  if (!coef || n == 0) {
    c->has_cal = false;
    return FR3D_OK;
  }
  if (n != MLP_IN + 1) return fail(c, FR3D_E_INVALID, "need %d calibration coefficients", MLP_IN + 1);
  for (int64_t i = 0; i < n; ++i)
    if (!std::isfinite(coef[i])) return fail(c, FR3D_E_INVALID, "calibration coefficients must be finite");
  if (!c->has_pred) return fail(c, FR3D_E_STATE, "no predictor loaded");
  if (!c->pred_cal) HIPCHK(c, hipMalloc(&c->pred_cal, (MLP_IN + 1) * sizeof(double)));
  hipStream_t st = c->lanes[0].stream;
  HIPCHK(c, hipMemcpyAsync(c->pred_cal, coef, (MLP_IN + 1) * sizeof(double), hipMemcpyHostToDevice, st));
  HIPCHK(c, hipStreamSynchronize(st));
  c->has_cal = true;
  return FR3D_OK;
}

fr3d_status fr3d_predictor_get(fr3d_ctx* c, float* params, float* norm) {
  if (!c) return FR3D_E_INVALID;
  if (!c->has_pred) return fail(c, FR3D_E_STATE, "no predictor loaded");
  hipStream_t st = c->lanes[0].stream;
  if (params) HIPCHK(c, hipMemcpyAsync(params, c->pred_p, MLP_NP * sizeof(float), hipMemcpyDeviceToHost, st));
  if (norm) HIPCHK(c, hipMemcpyAsync(norm, c->pred_norm, MLP_NNORM * sizeof(float), hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  return FR3D_OK;
}

fr3d_status fr3d_predictor_forward(fr3d_ctx* c, const float* X, int32_t B, float* y) {
  if (!c) return FR3D_E_INVALID;
  if (!c->has_pred) return fail(c, FR3D_E_STATE, "no predictor loaded");
  if (!X || !y || B <= 0) return fail(c, FR3D_E_INVALID, "need X, y and B > 0");
  LCHK(c, mlp_forward(c->pred_p, c->pred_norm, X, B, y, nullptr, nullptr, c->lanes[0].stream));
  return FR3D_OK;
}

fr3d_status fr3d_predictor_train_step(fr3d_ctx* c, const float* X, const float* t, int32_t B, double lr,
                                      float* loss, float* grad) {
  if (!c) return FR3D_E_INVALID;
  if (!c->has_pred) return fail(c, FR3D_E_STATE, "no predictor loaded");
  if (!X || !t || B <= 0 || B > 65536) return fail(c, FR3D_E_INVALID, "need X, t and 0 < B <= 65536");
  if (!(lr >= 0) || !std::isfinite(lr)) return fail(c, FR3D_E_INVALID, "lr must be finite and >= 0");
  fr3d_status s = pred_ensure_work(c, B);
  if (s) return s;
  MlpWork w;
  mlp_work_carve(&w, c->pred_work, c->pred_cap);
  hipStream_t st = c->lanes[0].stream;
  LCHK(c, mlp_forward(c->pred_p, c->pred_norm, X, B, nullptr, &w, nullptr, st));
  const long long step = lr > 0 ? c->pred_step + 1 : c->pred_step;
  const double c1 = 1.0 - std::pow(0.9, (double)std::max(1LL, step));
  const double c2 = 1.0 - std::pow(0.999, (double)std::max(1LL, step));
  LCHK(c, mlp_backward_adam(c->pred_p, c->pred_norm, t, B, &w, c->pred_g, c->pred_loss, c->pred_m, c->pred_v, lr, c1,
                            c2, st));
  if (lr > 0) c->pred_step = step;
  if (loss) HIPCHK(c, hipMemcpyAsync(loss, c->pred_loss, sizeof(float), hipMemcpyDeviceToDevice, st));
  if (grad) HIPCHK(c, hipMemcpyAsync(grad, c->pred_g, MLP_NP * sizeof(float), hipMemcpyDeviceToDevice, st));
  return FR3D_OK;
}

// File: "FR3DMLP1", int32 n_params, int32 n_norm, int64 step, params, norm,
// Adam m, Adam v (FP32 little-endian), uint64 FNV-1a of everything before it.
fr3d_status fr3d_predictor_save(fr3d_ctx* c, const char* path) {
  if (!c || !path) return FR3D_E_INVALID;
  if (!c->has_pred) return fail(c, FR3D_E_STATE, "no predictor loaded");
  std::vector<float> p(MLP_NP), nm(MLP_NNORM), m(MLP_NP), v(MLP_NP);
  hipStream_t st = c->lanes[0].stream;
  HIPCHK(c, hipMemcpyAsync(p.data(), c->pred_p, MLP_NP * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipMemcpyAsync(nm.data(), c->pred_norm, MLP_NNORM * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipMemcpyAsync(m.data(), c->pred_m, MLP_NP * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipMemcpyAsync(v.data(), c->pred_v, MLP_NP * 4, hipMemcpyDeviceToHost, st));
  HIPCHK(c, hipStreamSynchronize(st));
  std::string buf("FR3DMLP1");
  const int32_t np = MLP_NP, nn = MLP_NNORM;
  const int64_t step = c->pred_step;
  buf.append((const char*)&np, 4).append((const char*)&nn, 4).append((const char*)&step, 8);
  buf.append((const char*)p.data(), p.size() * 4).append((const char*)nm.data(), nm.size() * 4);
  buf.append((const char*)m.data(), m.size() * 4).append((const char*)v.data(), v.size() * 4);
  const uint64_t h = fnv1a(buf.data(), buf.size());
  buf.append((const char*)&h, 8);
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(c, FR3D_E_INVALID, "cannot open %s for writing", path);
  const size_t w = std::fwrite(buf.data(), 1, buf.size(), f);
  const int cl = std::fclose(f);
  if (w != buf.size() || cl != 0) return fail(c, FR3D_E_INVALID, "write to %s failed", path);
  return FR3D_OK;
}

fr3d_status fr3d_predictor_load(fr3d_ctx* c, const char* path) {
  if (!c || !path) return FR3D_E_INVALID;
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(c, FR3D_E_INVALID, "cannot open %s", path);
  std::string buf;
  char tmp[65536];
  size_t r;
  while ((r = std::fread(tmp, 1, sizeof tmp, f)) > 0) buf.append(tmp, r);
  std::fclose(f);
  const size_t want = 8 + 16 + (size_t)(3 * MLP_NP + MLP_NNORM) * 4 + 8;
  if (buf.size() != want || buf.compare(0, 8, "FR3DMLP1") != 0) return fail(c, FR3D_E_INVALID, "%s: not a predictor file", path);
  uint64_t h;
  std::memcpy(&h, buf.data() + buf.size() - 8, 8);
  if (h != fnv1a(buf.data(), buf.size() - 8)) return fail(c, FR3D_E_INVALID, "%s: checksum mismatch", path);
  int32_t np, nn;
  int64_t step;
  std::memcpy(&np, buf.data() + 8, 4);
  std::memcpy(&nn, buf.data() + 12, 4);
  std::memcpy(&step, buf.data() + 16, 8);
  if (np != MLP_NP || nn != MLP_NNORM) return fail(c, FR3D_E_INVALID, "%s: wrong network shape", path);
  std::vector<float> all((buf.size() - 32) / 4);
  std::memcpy(all.data(), buf.data() + 24, all.size() * 4);
  const float* p = all.data();
  const float* nm = p + MLP_NP;
  const float* m = nm + MLP_NNORM;
  const float* v = m + MLP_NP;
  fr3d_status s = fr3d_predictor_set(c, p, MLP_NP, nm);
  if (s) return s;
  hipStream_t st = c->lanes[0].stream;
  HIPCHK(c, hipMemcpyAsync(c->pred_m, m, MLP_NP * 4, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipMemcpyAsync(c->pred_v, v, MLP_NP * 4, hipMemcpyHostToDevice, st));
  HIPCHK(c, hipStreamSynchronize(st));
  c->pred_step = step;
  return FR3D_OK;
}

}  // extern "C"
