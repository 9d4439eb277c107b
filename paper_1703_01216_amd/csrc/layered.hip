// Kernels of Algorithm 1 with per-frequency z-systems (layouts in layered.hpp).
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include "layered.hpp"

namespace fr3d {

namespace {

constexpr int LNT = 256;   // threads per workgroup of the per-evaluation kernels
constexpr int SNT = 1024;  // threads of the SVD kernel: 16 waves share a round's column pairs

// Round-robin ("circle") pairing of n2 (even) columns: in round r, column 0
// meets c(0) and column c(p) meets c(n2 - 1 - p), with c(k) = 1 + (k + r) mod (n2 - 1).
__device__ __forceinline__ void rr_pair(int r, int p, int n2, int& i, int& j) {
  const int m = n2 - 1;
  if (p == 0) {
    i = 0;
    j = 1 + r % m;
  } else {
    i = 1 + (p + r) % m;
    j = 1 + (n2 - 1 - p + r) % m;
  }
}

// One workgroup per distinct system: A from the Toeplitz entries, then
// one-sided Jacobi (Hestenes) rotations on pairs of columns until every pair
// is orthogonal to 1e-15 relative (at most 40 sweeps); the rotated columns'
// squared norms are s_k^2 and the accumulated rotations are V.
__global__ __launch_bounds__(SNT) void k_lay_svd(const double2* __restrict__ Bk, LayArgs la, double* __restrict__ kt,
                                                  double* __restrict__ V, double* __restrict__ lam) {
  __shared__ double As[LAY_MMAX * LAY_MMAX];  // column j at j*M
  __shared__ double Vs[LAY_MMAX * LAY_MMAX];  // column k at k*M
  __shared__ double ktv[2 * LAY_MMAX];
  __shared__ double offw[SNT / 64];
  const int M = la.M, L = 2 * M - 1;
  const int f = blockIdx.x;
  const int kx = f / la.pyh, my = f % la.pyh;
  const int tid = threadIdx.x, w = tid / 64, lane = tid % 64;
  for (int l = tid; l < L; l += SNT) {
    const double v = Bk[((size_t)kx * L + l) * la.py + my].x;
    ktv[l] = v;
    kt[(size_t)f * L + l] = v;
  }
  __syncthreads();
  for (int e = tid; e < M * M; e += SNT) {
    const int i = e % M, j = e / M;
    As[e] = ktv[i - j + M - 1];
    Vs[e] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  const int n2 = M + (M & 1);
  const double tol = 1e-15;
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0;
    for (int r = 0; r < n2 - 1; ++r) {
      for (int p = w; p < n2 / 2; p += SNT / 64) {
        int i, j;
        rr_pair(r, p, n2, i, j);
        if (i >= M || j >= M) continue;  // the dummy column of an odd M
        const double ai = lane < M ? As[i * M + lane] : 0.0;
        const double aj = lane < M ? As[j * M + lane] : 0.0;
        const double al = wave_sum<double>(ai * ai);
        const double be = wave_sum<double>(aj * aj);
        const double ga = wave_sum<double>(ai * aj);
        const double nrm = sqrt(al * be);
        if (!(fabs(ga) > tol * nrm) || ga == 0.0) continue;
        off = fmax(off, fabs(ga) / nrm);
        const double zeta = (be - al) / (2.0 * ga);
        const double t = copysign(1.0, zeta) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
        const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
        if (lane < M) {
          As[i * M + lane] = c * ai - s * aj;
          As[j * M + lane] = s * ai + c * aj;
          const double vi = Vs[i * M + lane], vj = Vs[j * M + lane];
          Vs[i * M + lane] = c * vi - s * vj;
          Vs[j * M + lane] = s * vi + c * vj;
        }
      }
      __syncthreads();
    }
    if (lane == 0) offw[w] = off;
    __syncthreads();
    double mx = 0.0;
    for (int k = 0; k < SNT / 64; ++k) mx = fmax(mx, offw[k]);
    __syncthreads();
    if (mx <= tol) break;
  }
  for (int k = w; k < M; k += SNT / 64) {
    const double a = lane < M ? As[k * M + lane] : 0.0;
    const double s2 = wave_sum<double>(a * a);
    if (lane == 0) lam[(size_t)f * M + k] = s2;
  }
  double* Vf = V + (size_t)f * M * M;
  for (int e = tid; e < M * M; e += SNT) {
    const int i = e / M, k = e % M;
    Vf[e] = Vs[k * M + i];
  }
}

__device__ __forceinline__ double lay_gain(int filt, int order, double lam, double a) {
  if (filt == 0) return 1.0 / (lam + a);
  if (filt == 1) {
    const double d = 1.0 / (lam + a), q = a * d;
    double qp = 1.0, sum = 1.0;
    for (int j = 1; j < order; ++j) {
      qp *= q;
      sum += qp;
    }
    return d * sum;
  }
  return lam >= a ? 1.0 / lam : 0.0;
}

// One workgroup per distinct system, serving the frequencies ky = |ky| and
// Py - |ky| (same A).  Mode 0 (search): w = A^T f^, b = V^T w, then for each
// candidate x^ = V (h b), r^ = A x^ - f^ written as (x^, r^) pairs; mode 1
// (forward operator): (A x^, 0), or (A^T x^, 0) with a.adj.  FP64
// arithmetic, T in and out.
template <typename T, int MODE, bool KM>
__global__ __launch_bounds__(LNT) void k_lay_filter(const c2<T>* __restrict__ B, c4<T>* __restrict__ W1, LayArgs la,
                                                     InvArgs a) {
  __shared__ double Vs[LAY_MMAX * LAY_MMAX];  // V[i][k] at i*M + k
  __shared__ double ls[LAY_MMAX];
  __shared__ double ktv[2 * LAY_MMAX];
  __shared__ double2 fs[2][LAY_MMAX], ws[2][LAY_MMAX], hb[2][LAY_MMAX], xs[2][LAY_MMAX];
  if (inv_idle(a)) return;
  int cb = 0, ce = 1;
  if constexpr (KM) {
    cb = blockIdx.y * a.kb;
    ce = min(cb + a.kb, a.ctrl->kc);
    if (cb >= ce) return;
    W1 = (c4<T>*)a.ctrl->kw1;  // the search's K-candidate workspace
  }
  const int M = la.M, L = 2 * M - 1;
  const int f = blockIdx.x;
  const int kx = f / la.pyh, my = f % la.pyh;
  const int nky = (my > 0 && 2 * my != la.py) ? 2 : 1;
  const int tid = threadIdx.x;
  for (int l = tid; l < L; l += LNT) ktv[l] = la.kt[(size_t)f * L + l];
  if constexpr (MODE == 0) {
    // all of the system's V in flight at once (up to 15 loads per thread), then to LDS
    constexpr int NV = (LAY_MMAX * LAY_MMAX + LNT - 1) / LNT;
    const double* Vf = la.V + (size_t)f * M * M;
    const int MM = M * M;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e = tid + k * LNT;
      v[k] = e < MM ? Vf[e] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e = tid + k * LNT;
      if (e < MM) Vs[e] = v[k];
    }
    for (int k = tid; k < M; k += LNT) ls[k] = la.lam[(size_t)f * M + k];
  }
  for (int e = tid; e < nky * M; e += LNT) {
    const int q = e / M, i = e % M;
    const int ky = q == 0 ? my : la.py - my;
    const c2<T> v = B[((size_t)kx * M + i) * la.py + ky];
    fs[q][i] = make_double2((double)v.x, (double)v.y);
  }
  __syncthreads();
  const int q = tid / 128, i = tid % 128;  // system copy (ky) and row of this thread
  const bool act = q < nky && i < M;
  const int ky = q == 0 ? my : la.py - my;
  if constexpr (MODE == 1) {
    if (act) {
      double2 y = make_double2(0.0, 0.0);
      for (int j = 0; j < M; ++j) {
        const double k = a.adj ? ktv[j - i + M - 1] : ktv[i - j + M - 1];  // A^T or A
        y.x += k * fs[q][j].x;
        y.y += k * fs[q][j].y;
      }
      c4<T> o;
      o.x = (T)y.x; o.y = (T)y.y; o.z = (T)0; o.w = (T)0;
      W1[((size_t)kx * M + i) * la.py + ky] = o;
    }
    return;
  } else {
    if (act) {  // w = A^T f
      double2 s = make_double2(0.0, 0.0);
      for (int r = 0; r < M; ++r) {
        const double k = ktv[r - i + M - 1];
        s.x += k * fs[q][r].x;
        s.y += k * fs[q][r].y;
      }
      ws[q][i] = s;
    }
    __syncthreads();
    double2 bk = make_double2(0.0, 0.0);  // b = V^T w, thread i holds b_i
    if (act) {
      for (int r = 0; r < M; ++r) {
        const double v = Vs[r * M + i];
        bk.x += v * ws[q][r].x;
        bk.y += v * ws[q][r].y;
      }
    }
    for (int cand = cb; cand < ce; ++cand) {
      const double aa = KM ? a.ctrl->ca[cand] : a.ctrl->alpha_abs;
      if (act) {
        const double h = lay_gain(a.filt, a.order, ls[i], aa);
        hb[q][i] = make_double2(h * bk.x, h * bk.y);
      }
      __syncthreads();
      if (act) {  // x = V (h b)
        double2 x = make_double2(0.0, 0.0);
        for (int k = 0; k < M; ++k) {
          const double v = Vs[i * M + k];
          x.x += v * hb[q][k].x;
          x.y += v * hb[q][k].y;
        }
        xs[q][i] = x;
      }
      __syncthreads();
      if (act) {  // r = A x - f
        double2 r = make_double2(-fs[q][i].x, -fs[q][i].y);
        for (int j = 0; j < M; ++j) {
          const double k = ktv[i - j + M - 1];
          r.x += k * xs[q][j].x;
          r.y += k * xs[q][j].y;
        }
        c4<T> o;
        o.x = (T)xs[q][i].x; o.y = (T)xs[q][i].y; o.z = (T)r.x; o.w = (T)r.y;
        W1[(KM ? (size_t)cand * a.w1_stride : 0) + ((size_t)kx * M + i) * la.py + ky] = o;
      }
      __syncthreads();
    }
  }
}

// Per-frequency alphas (see layered.hpp).  Wave 2q runs the search of the
// system copy q (ky or Py - ky); the other waves wait at the barrier.
template <typename T>
__global__ __launch_bounds__(LNT) void k_lay_pf(const c2<T>* __restrict__ B, c4<T>* __restrict__ W1, LayArgs la,
                                                 InvArgs a, PfArgs pf) {
  __shared__ double Vs[LAY_MMAX * LAY_MMAX];
  __shared__ double ls[LAY_MMAX];
  __shared__ double ktv[2 * LAY_MMAX];
  __shared__ double2 fs[2][LAY_MMAX], ws[2][LAY_MMAX], hb[2][LAY_MMAX], xs[2][LAY_MMAX];
  __shared__ double b2[2][LAY_MMAX];
  __shared__ double alph[2], tsel[2];
  __shared__ int flg[2];
  if (inv_idle(a)) return;
  const int M = la.M, L = 2 * M - 1;
  const int f = blockIdx.x;
  const int kx = f / la.pyh, my = f % la.pyh;
  const int nky = (my > 0 && 2 * my != la.py) ? 2 : 1;
  const int tid = threadIdx.x;
  for (int l = tid; l < L; l += LNT) ktv[l] = la.kt[(size_t)f * L + l];
  {
    constexpr int NV = (LAY_MMAX * LAY_MMAX + LNT - 1) / LNT;
    const double* Vf = la.V + (size_t)f * M * M;
    const int MM = M * M;
    double v[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e = tid + k * LNT;
      v[k] = e < MM ? Vf[e] : 0.0;
    }
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      const int e = tid + k * LNT;
      if (e < MM) Vs[e] = v[k];
    }
  }
  for (int k = tid; k < M; k += LNT) ls[k] = la.lam[(size_t)f * M + k];
  for (int e = tid; e < nky * M; e += LNT) {
    const int q = e / M, i = e % M;
    const int ky = q == 0 ? my : la.py - my;
    const c2<T> v = B[((size_t)kx * M + i) * la.py + ky];
    fs[q][i] = make_double2((double)v.x, (double)v.y);
  }
  __syncthreads();
  const int q = tid / 128, i = tid % 128;
  const bool act = q < nky && i < M;
  const int ky = q == 0 ? my : la.py - my;
  if (act) {  // w = A^T f
    double2 s = make_double2(0.0, 0.0);
    for (int r = 0; r < M; ++r) {
      const double k = ktv[r - i + M - 1];
      s.x += k * fs[q][r].x;
      s.y += k * fs[q][r].y;
    }
    ws[q][i] = s;
  }
  __syncthreads();
  double2 bk = make_double2(0.0, 0.0);  // b = V^T w
  if (act) {
    for (int r = 0; r < M; ++r) {
      const double v = Vs[r * M + i];
      bk.x += v * ws[q][r].x;
      bk.y += v * ws[q][r].y;
    }
    b2[q][i] = bk.x * bk.x + bk.y * bk.y;
  }
  __syncthreads();
  if (i < 64 && q < nky) {  // the search, one wave per system copy
    const int lane = i;
    double ff = 0.0;
    for (int k = lane; k < M; k += 64) ff += fs[q][k].x * fs[q][k].x + fs[q][k].y * fs[q][k].y;
    ff = wave_sum<double>(ff);
    const double T2 = pf.target * pf.target;
    auto rho_ratio = [&](double t, double& rho, double& ratio) {
      const double aa = pow(10.0, t) * pf.a_scale;
      double s = 0.0;
      for (int k = lane; k < M; k += 64) {
        const double lam = ls[k];
        const double h = lay_gain(a.filt, a.order, lam, aa);
        s += (2.0 * h - lam * h * h) * b2[q][k];
      }
      s = wave_sum<double>(s);
      const double r2 = fmax(ff - s, 0.0);
      rho = r2 - T2;
      ratio = T2 > 0 ? sqrt(r2) / pf.target : INFINITY;
    };
    double rho, ratio, t = pf.hi;
    int fl = 0;
    bool done = false;
    rho_ratio(pf.hi, rho, ratio);
    if (fabs(ratio - 1.0) <= pf.tol) done = true;
    else if (rho < 0) { fl = F_NOROOT_HIGH; done = true; }
    if (!done) {
      t = pf.lo;
      rho_ratio(pf.lo, rho, ratio);
      if (fabs(ratio - 1.0) <= pf.tol) done = true;
      else if (rho > 0) { fl = F_NOROOT_LOW; done = true; }
    }
    if (!done) {
      double lo = pf.lo, hi = pf.hi;
      for (int st = 0; st < pf.max_steps && !done; ++st) {
        t = 0.5 * (lo + hi);
        rho_ratio(t, rho, ratio);
        if (fabs(ratio - 1.0) <= pf.tol) done = true;
        else if (rho < 0) lo = t;
        else hi = t;
      }
      if (!done) { t = hi; fl = F_MAXITER; }
    }
    if (lane == 0) {
      tsel[q] = t;
      alph[q] = pow(10.0, t) * pf.a_scale;
      flg[q] = fl;
    }
  }
  __syncthreads();
  if (act) {
    const double h = lay_gain(a.filt, a.order, ls[i], alph[q]);
    hb[q][i] = make_double2(h * bk.x, h * bk.y);
  }
  __syncthreads();
  if (act) {  // x = V (h b)
    double2 x = make_double2(0.0, 0.0);
    for (int k = 0; k < M; ++k) {
      const double v = Vs[i * M + k];
      x.x += v * hb[q][k].x;
      x.y += v * hb[q][k].y;
    }
    xs[q][i] = x;
  }
  __syncthreads();
  if (act) {  // r = A x - f
    double2 r = make_double2(-fs[q][i].x, -fs[q][i].y);
    for (int j = 0; j < M; ++j) {
      const double k = ktv[i - j + M - 1];
      r.x += k * xs[q][j].x;
      r.y += k * xs[q][j].y;
    }
    c4<T> o;
    o.x = (T)xs[q][i].x; o.y = (T)xs[q][i].y; o.z = (T)r.x; o.w = (T)r.y;
    W1[((size_t)kx * M + i) * la.py + ky] = o;
  }
  if (tid == 0) {
    // counts over the full Px x Py spectrum: columns 0 < kx < Px/2 stand for
    // their mirror images too
    const double wx = (kx > 0 && kx != la.kxn - 1) ? 2.0 : 1.0;
    double sl = 0.0, nh = 0.0, nl = 0.0, nm = 0.0;
    for (int c = 0; c < nky; ++c) {
      sl += wx * tsel[c];
      nh += wx * (flg[c] == F_NOROOT_HIGH);
      nl += wx * (flg[c] == F_NOROOT_LOW);
      nm += wx * (flg[c] == F_MAXITER);
      const int kyc = c == 0 ? my : la.py - my;
      if (pf.alpha_out) pf.alpha_out[(size_t)kx * la.py + kyc] = pow(10.0, tsel[c]);
      if (pf.flags_out) pf.flags_out[(size_t)kx * la.py + kyc] = flg[c];
    }
    double* pp = pf.part + (size_t)5 * f;
    pp[0] = sl;
    pp[1] = wx * nky;
    pp[2] = nh;
    pp[3] = nl;
    pp[4] = nm;
  }
}

// One thread per system: the squared singular values to singular values,
// sorted descending by insertion (M <= 60).
__global__ __launch_bounds__(LNT) void k_lay_sv(LayArgs la, double* __restrict__ out) {
  const long long f = (long long)blockIdx.x * LNT + threadIdx.x;
  if (f >= (long long)la.kxn * la.pyh) return;
  const int M = la.M;
  const double* lam = la.lam + (size_t)f * M;
  double* o = out + (size_t)f * M;
  for (int k = 0; k < M; ++k) {
    const double v = sqrt(fmax(lam[k], 0.0));
    int j = k;
    while (j > 0 && o[j - 1] < v) {
      o[j] = o[j - 1];
      --j;
    }
    o[j] = v;
  }
}

__global__ __launch_bounds__(LNT) void k_lay_max_part(const double* __restrict__ lam, long long n, double* part) {
  __shared__ double red[LNT / 64];
  double m = 0.0;
  for (long long e = blockIdx.x * (long long)LNT + threadIdx.x; e < n; e += (long long)gridDim.x * LNT)
    m = fmax(m, lam[e]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < LNT / 64; ++k) t = fmax(t, red[k]);
    part[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(LNT) void k_lay_max_final(const double* __restrict__ part, int n, double* out) {
  __shared__ double red[LNT / 64];
  double m = 0.0;
  for (int e = threadIdx.x; e < n; e += LNT) m = fmax(m, part[e]);
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
  if (threadIdx.x % 64 == 0) red[threadIdx.x / 64] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int k = 0; k < LNT / 64; ++k) t = fmax(t, red[k]);
    *out = t;
  }
}

template <typename K, typename... Args>
hipError_t go_lay(K kern, dim3 g, const Launch& L, Args... args) {
  if (L.e0) hipExtLaunchKernelGGL(kern, g, dim3(LNT), 0, L.s, L.e0, L.e1, 0, args...);
  else hipLaunchKernelGGL(kern, g, dim3(LNT), 0, L.s, args...);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_lay_svd(const double2* Bk, const LayArgs& la, double* kt, double* V, double* lam, hipStream_t s) {
  if (la.M < 1 || la.M > LAY_MMAX) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_lay_svd, dim3((unsigned)(la.kxn * la.pyh)), dim3(SNT), 0, s, Bk, la, kt, V, lam);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lay_filter(int mode, const c2<T>* B, c4<T>* W1, const LayArgs& la, const InvArgs& a,
                             const Launch& L) {
  if (la.M < 1 || la.M > LAY_MMAX) return hipErrorInvalidValue;
  dim3 g((unsigned)(la.kxn * la.pyh));
  if (mode != 0) return go_lay(k_lay_filter<T, 1, false>, g, L, B, W1, la, a);
  if (a.kmode) {
    g.y = (unsigned)((a.kmax + a.kb - 1) / a.kb);
    return go_lay(k_lay_filter<T, 0, true>, g, L, B, W1, la, a);
  }
  return go_lay(k_lay_filter<T, 0, false>, g, L, B, W1, la, a);
}

hipError_t launch_lay_sv(const LayArgs& la, double* out, hipStream_t s) {
  const long long nf = (long long)la.kxn * la.pyh;
  hipLaunchKernelGGL(k_lay_sv, dim3((unsigned)((nf + LNT - 1) / LNT)), dim3(LNT), 0, s, la, out);
  return hipGetLastError();
}

hipError_t launch_lay_max(const double* lam, long long n, double* part, double* out, hipStream_t s) {
  const unsigned nb = (unsigned)std::min<long long>((n + LNT - 1) / LNT, 1024);
  hipLaunchKernelGGL(k_lay_max_part, dim3(nb), dim3(LNT), 0, s, lam, n, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_lay_max_final, dim3(1), dim3(LNT), 0, s, (const double*)part, (int)nb, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_lay_pf(const c2<T>* B, c4<T>* W1, const LayArgs& la, const InvArgs& a, const PfArgs& pf,
                         const Launch& L) {
  if (la.M < 1 || la.M > LAY_MMAX) return hipErrorInvalidValue;
  return go_lay(k_lay_pf<T>, dim3((unsigned)(la.kxn * la.pyh)), L, B, W1, la, a, pf);
}

template hipError_t launch_lay_pf<float>(const c2<float>*, c4<float>*, const LayArgs&, const InvArgs&,
                                         const PfArgs&, const Launch&);
template hipError_t launch_lay_pf<double>(const c2<double>*, c4<double>*, const LayArgs&, const InvArgs&,
                                          const PfArgs&, const Launch&);
template hipError_t launch_lay_filter<float>(int, const c2<float>*, c4<float>*, const LayArgs&, const InvArgs&,
                                             const Launch&);
template hipError_t launch_lay_filter<double>(int, const c2<double>*, c4<double>*, const LayArgs&, const InvArgs&,
                                              const Launch&);

}  // namespace fr3d
