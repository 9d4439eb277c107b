// Pass kernels of the padded 3D transforms (layouts in passes.hpp).  Included
// by one translation unit per precision, which instantiates the launchers.
#pragma once
#include "passes.hpp"

namespace fr3d {

// ============================================================ forward x pass
// Real-to-complex transform along x.  Two real rows share one complex pencil
// (a + i b); after the transform A(k) = (Z(k) + conj Z(P-k))/2 and
// B(k) = (Z(k) - conj Z(P-k))/(2i).  Data mode reads the n = P/2 valid
// samples of each row; generator mode samples the kernel's offset table on
// the fly (Sec. 3 kernel, Sec. 5 midpoint weight h^3; the slot at offset
// index n is zero).
__device__ __forceinline__ double kernel_value(int kind, double x, double y, double z) {
  const double r2 = x * x + y * y + z * z;
  const double rr = sqrt(r2);
  return kind == 0 ? -z / (r2 * rr) : 1.0 / rr;
}

__device__ __forceinline__ bool wrap_offset(int a, int n, int p, int& off) {
  if (a < n) { off = a; return true; }
  if (a > p - n) { off = a - p; return true; }
  return false;
}

template <typename T, int P, bool GEN>
__global__ __launch_bounds__(NT) void k_fx(const T* __restrict__ F, c2<T>* __restrict__ A, FwdArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int C = Tile<T, P>::C;  // complex pencils per tile = C, real rows = 2C
  constexpr int LD = P + 1;
  constexpr int N = P / 2;
  __shared__ c2<T> lds[C * LD];
  __shared__ c2<T> tw[P];
  const int tid = threadIdx.x;
  const int z = blockIdx.y;
  const int y0 = blockIdx.x * (2 * C);
  load_twiddles<T, P, NT>(tw, twg, tid);
  T* ldsr = reinterpret_cast<T*>(lds);
  if constexpr (!GEN) {
    // rows y0 .. y0+2C-1 of plane z are contiguous: 2C*N floats
    const int rows = min(2 * C, a.ny_in - y0);
    const T* src = F + ((size_t)z * a.ny_in + y0) * N;
    for (int e = tid; e < 2 * C * N; e += NT) {
      const int r = e / N, x = e % N;
      const T v = r < rows ? src[e] : (T)0;
      ldsr[2 * ((r >> 1) * LD + x) + (r & 1)] = v;
    }
    for (int e = tid; e < C * (P - N); e += NT) {
      const int c = e / (P - N), x = N + e % (P - N);
      lds[c * LD + x] = mk<T>(0, 0);
    }
  } else {
    for (int e = tid; e < 2 * C * P; e += NT) {
      const int r = e / P, x = e % P;
      const int yb = y0 + r;
      double v = 0.0;
      int ox, oy, oz;
      if (yb < a.ny_in && wrap_offset(x, a.nx, P, ox) && wrap_offset(yb, a.ny, a.py, oy) &&
          wrap_offset(z, a.nz, a.pz, oz)) {
        v = a.h * a.h * a.h * kernel_value(a.kind, ox * a.h, oy * a.h, (a.D + oz) * a.h);
      }
      ldsr[2 * ((r >> 1) * LD + x) + (r & 1)] = (T)v;
    }
  }
  __syncthreads();
  tile_fft<T, P, C, LD, NT, false, -1>(lds, tw, tid);
  const int kxn = P / 2 + 1;
  for (int e = tid; e < kxn * 2 * C; e += NT) {
    const int yl = e % (2 * C), kx = e / (2 * C);
    const int y = y0 + yl;
    if (y >= a.ny_in) continue;
    const int c = yl >> 1;
    const c2<T> Z = lds[c * LD + kx];
    const c2<T> Zm = lds[c * LD + (P - kx) % P];
    c2<T> v;
    if ((yl & 1) == 0) v = mk<T>((T)0.5 * (Z.x + Zm.x), (T)0.5 * (Z.y - Zm.y));
    else v = mk<T>((T)0.5 * (Z.y + Zm.y), (T)0.5 * (Zm.x - Z.x));
    A[((size_t)kx * a.nz_in + z) * a.ny_in + y] = v;
  }
}

// ============================================================ forward y pass
// Complex transform along y of every row (kx, z); rows are contiguous.
template <typename T, int P, bool PRUNE>
__global__ __launch_bounds__(NT) void k_fy(const c2<T>* __restrict__ A, c2<T>* __restrict__ B, FwdArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int C = Tile<T, P>::C;
  constexpr int LD = P + 1;
  constexpr int NIN = PRUNE ? P / 2 : P;
  __shared__ c2<T> lds[C * LD];
  __shared__ c2<T> tw[P];
  const int tid = threadIdx.x;
  const long long nrows = (long long)a.kx_n * a.nz_in;
  const long long row0 = (long long)blockIdx.x * C;
  const int rows = (int)min((long long)C, nrows - row0);
  load_twiddles<T, P, NT>(tw, twg, tid);
  const c2<T>* src = A + row0 * NIN;
  for (int e = tid; e < C * NIN; e += NT) {
    const int r = e / NIN, y = e % NIN;
    lds[r * LD + y] = r < rows ? src[e] : mk<T>(0, 0);
  }
  if constexpr (PRUNE) {
    for (int e = tid; e < C * (P - NIN); e += NT) {
      const int r = e / (P - NIN), y = NIN + e % (P - NIN);
      lds[r * LD + y] = mk<T>(0, 0);
    }
  }
  __syncthreads();
  tile_fft<T, P, C, LD, NT, false, -1>(lds, tw, tid);
  c2<T>* dst = B + row0 * P;
  for (int e = tid; e < rows * P; e += NT) {
    const int r = e / P, y = e % P;
    dst[e] = lds[r * LD + y];
  }
}

// ============================================================ forward z pass
// Complex transform along z of C consecutive ky-columns of one kx plane.
// MODE 0 (data): n inputs, P outputs, fused radial-energy epilogue whose last
// workgroup also forms the predictor features.  MODE 1 (kernel spectrum): P
// inputs, only kz <= P/2 and ky <= Py/2 stored (the octant).
template <typename T, int P, int MODE>
__global__ __launch_bounds__(NT) void k_fz(const c2<T>* __restrict__ B, c2<T>* __restrict__ S, FwdArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int C = Tile<T, P>::C;
  constexpr int LD = C;
  constexpr int NIN = MODE == 0 ? P / 2 : P;
  constexpr int NOUT = MODE == 0 ? P : P / 2 + 1;
  __shared__ c2<T> lds[P * LD];
  __shared__ c2<T> tw[P];
  __shared__ double bins[64];
  __shared__ int last;
  const int tid = threadIdx.x;
  const int kx = blockIdx.y;
  const int ky0 = blockIdx.x * C;
  const int py = a.py;
  load_twiddles<T, P, NT>(tw, twg, tid);
  if (MODE == 0 && tid < 64) bins[tid] = 0.0;
  const c2<T>* src = B + (size_t)kx * NIN * py;
  for (int e = tid; e < C * NIN; e += NT) {
    const int z = e / C, col = e % C;
    const int ky = ky0 + col;
    lds[z * LD + col] = ky < py ? src[(size_t)z * py + ky] : mk<T>(0, 0);
  }
  if constexpr (NIN < P) {
    for (int e = tid; e < C * (P - NIN); e += NT) lds[NIN * LD + e] = mk<T>(0, 0);
  }
  __syncthreads();
  tile_fft<T, P, C, LD, NT, true, -1>(lds, tw, tid);
  if constexpr (MODE == 0) {
    c2<T>* dst = S + (size_t)kx * P * py;
    const double w = (kx == 0 || 2 * kx == a.bg.px) ? 1.0 : 2.0;
    int cur = -1;
    double acc = 0.0;
    for (int e = tid; e < C * P; e += NT) {
      const int kz = e / C, col = e % C;
      const int ky = ky0 + col;
      if (ky >= py) continue;
      const c2<T> v = lds[kz * LD + col];
      dst[(size_t)kz * py + ky] = v;
      const int b = energy_bin(a.bg, kx, ky, kz);
      if (b != cur) {
        if (cur >= 0) atomicAdd(&bins[cur], acc);
        cur = b;
        acc = 0.0;
      }
      acc += w * ((double)v.x * v.x + (double)v.y * v.y);
    }
    if (cur >= 0) atomicAdd(&bins[cur], acc);
    __syncthreads();
    const int nblk = gridDim.x * gridDim.y;
    const int bid = blockIdx.y * gridDim.x + blockIdx.x;
    if (tid < 64) a.bins_part[(size_t)bid * 64 + tid] = bins[tid];
    __threadfence();
    __syncthreads();
    if (tid == 0) last = (atomicAdd(a.ticket, 1u) == (unsigned)(nblk - 1));
    __syncthreads();
    if (!last) return;
    __threadfence();
    // deterministic final sum: bin = tid & 63, four partial lanes per bin
    double s = 0.0;
    const int bin = tid & 63, part = tid >> 6;
    for (int k = part; k < nblk; k += NT / 64)
      s += __hip_atomic_load(&a.bins_part[(size_t)k * 64 + bin], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (part == 0) bins[bin] = 0.0;
    __syncthreads();
    for (int p = 0; p < NT / 64; ++p) {
      if (part == p) bins[bin] += s;
      __syncthreads();
    }
    if (tid < 64) a.bins_out[tid] = bins[tid];
    if (tid == 0) {
      double tot = 0.0;
      for (int b = 0; b < 64; ++b) tot += bins[b];
      const double mean = tot / 64.0;
      for (int b = 0; b < 64; ++b) a.feat_out[b] = (float)log10(bins[b] / mean + 1e-30);
      const double fnorm = sqrt(tot / ((double)a.bg.px * a.bg.py * a.bg.pz));
      a.feat_out[64] = (float)log10(a.delta / fnorm);
      *a.ticket = 0u;
    }
  } else {
    const int oy = py / 2 + 1;
    c2<T>* dst = S + (size_t)kx * NOUT * oy;
    for (int e = tid; e < C * NOUT; e += NT) {
      const int kz = e / C, col = e % C;
      const int ky = ky0 + col;
      if (ky < oy) dst[(size_t)kz * oy + ky] = lds[kz * LD + col];
    }
  }
}

// ============================================================ inverse z pass
// Reads f^ for C ky-columns of one kx plane and all kz, forms per point (FP64
// coefficients from the octant of k^, rounded to T):
//   MODE 0: u^ = conj(k^) f^ / (s + a),  r^ = -a f^ / (s + a)   (Tikhonov, s = |k^|^2)
//   MODE 1: u^ = k^ f^,  r^ = 0                                  (forward operator)
// transforms both along z and writes z < nz as (u, r) pairs.
template <typename T, int P, int MODE>
__global__ __launch_bounds__(NT) void k_iz(const c2<T>* __restrict__ S, c4<T>* __restrict__ W1, InvArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int C = Tile<T, P>::C / 2 > 0 ? Tile<T, P>::C / 2 : 1;
  constexpr int NC = 2 * C;
  constexpr int LD = NC;
  constexpr int NOUT = P / 2;
  __shared__ c2<T> lds[P * LD];
  __shared__ c2<T> tw[P];
  if (a.ctrl && !a.ctrl->active) return;
  const double aa = MODE == 0 ? a.ctrl->alpha_abs : 0.0;
  const int tid = threadIdx.x;
  const int kx = blockIdx.y;
  const int ky0 = blockIdx.x * C;
  const int py = a.py;
  const int oz = P / 2 + 1, oy = py / 2 + 1;
  load_twiddles<T, P, NT>(tw, twg, tid);
  const c2<T>* src = S + (size_t)kx * P * py;
  const double2* oc = a.oct + (size_t)kx * oz * oy;
  for (int e = tid; e < C * P; e += NT) {
    const int kz = e / C, col = e % C;
    const int ky = ky0 + col;
    c2<T> u = mk<T>(0, 0), r = mk<T>(0, 0);
    if (ky < py) {
      const c2<T> f = src[(size_t)kz * py + ky];
      const int mz = kz <= P / 2 ? kz : P - kz;
      const int my = ky <= py / 2 ? ky : py - ky;
      double2 k = oc[(size_t)mz * oy + my];
      if (kz > P / 2) k.y = -k.y;
      const double fx = (double)f.x, fy = (double)f.y;
      if constexpr (MODE == 0) {
        const double s = k.x * k.x + k.y * k.y;
        const double d = 1.0 / (s + aa);
        const double cx = k.x * d, cy = -k.y * d;  // conj(k^) / (s + a)
        u = mk<T>((T)(fx * cx - fy * cy), (T)(fx * cy + fy * cx));
        const double cr = -aa * d;
        r = mk<T>((T)(fx * cr), (T)(fy * cr));
      } else {
        u = mk<T>((T)(fx * k.x - fy * k.y), (T)(fx * k.y + fy * k.x));
      }
    }
    lds[kz * LD + col] = u;
    lds[kz * LD + C + col] = r;
  }
  __syncthreads();
  tile_fft<T, P, NC, LD, NT, true, +1>(lds, tw, tid);
  c4<T>* dst = W1 + (size_t)kx * NOUT * py;
  for (int e = tid; e < C * NOUT; e += NT) {
    const int z = e / C, col = e % C;
    const int ky = ky0 + col;
    if (ky >= py) continue;
    const c2<T> u = lds[z * LD + col], r = lds[z * LD + C + col];
    c4<T> v;
    v.x = u.x; v.y = u.y; v.z = r.x; v.w = r.y;
    dst[(size_t)z * py + ky] = v;
  }
}

// ============================================================ inverse y pass
// Rows (kx, z) of (u, r) pairs: both transformed along y, y < ny written.
template <typename T, int P>
__global__ __launch_bounds__(NT) void k_iy(const c4<T>* __restrict__ W1, c4<T>* __restrict__ W2, InvArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int C = Tile<T, P>::C / 2 > 0 ? Tile<T, P>::C / 2 : 1;  // rows per tile
  constexpr int NC = 2 * C;
  constexpr int LD = P + 1;
  constexpr int NOUT = P / 2;
  __shared__ c2<T> lds[NC * LD];
  __shared__ c2<T> tw[P];
  if (a.ctrl && !a.ctrl->active) return;
  const int tid = threadIdx.x;
  const long long nrows = (long long)a.kx_n * a.nz;
  const long long row0 = (long long)blockIdx.x * C;
  const int rows = (int)min((long long)C, nrows - row0);
  load_twiddles<T, P, NT>(tw, twg, tid);
  const c4<T>* src = W1 + row0 * P;
  for (int e = tid; e < C * P; e += NT) {
    const int r = e / P, y = e % P;
    c4<T> v;
    if (r < rows) v = src[e];
    else { v.x = v.y = v.z = v.w = (T)0; }
    lds[(2 * r) * LD + y] = mk<T>(v.x, v.y);
    lds[(2 * r + 1) * LD + y] = mk<T>(v.z, v.w);
  }
  __syncthreads();
  tile_fft<T, P, NC, LD, NT, false, +1>(lds, tw, tid);
  c4<T>* dst = W2 + row0 * NOUT;
  for (int e = tid; e < rows * NOUT; e += NT) {
    const int r = e / NOUT, y = e % NOUT;
    const c2<T> u = lds[(2 * r) * LD + y], w = lds[(2 * r + 1) * LD + y];
    c4<T> v;
    v.x = u.x; v.y = u.y; v.z = w.x; v.w = w.y;
    dst[e] = v;
  }
}

// ============================================================ inverse x pass
// For C consecutive y of one z: u and r are Hermitian in kx (their 3D
// transforms are real), so Z(kx) = U(kx) + i R(kx) over the full kx range
// (Z(P-kx) = conj U(kx) + i conj R(kx)) transforms to u + i r.  Writes
// zeta = Re/P^3 on R (MODE 0 and 1) and accumulates ||zeta||^2 and
// ||r||^2 = sum (Im/P^3)^2 in FP64; the last workgroup sums the partials in
// a fixed order and advances the alpha search (MODE 0).
template <typename T, int P, int MODE>
__global__ __launch_bounds__(NT) void k_ix(const c4<T>* __restrict__ W2, T* __restrict__ out, InvArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int C = Tile<T, P>::C;
  constexpr int LD = C + 1;
  constexpr int NOUT = P / 2;
  constexpr int KXN = P / 2 + 1;
  __shared__ c2<T> lds[P * LD];
  __shared__ c2<T> tw[P];
  __shared__ double red[NT / 64];
  __shared__ int last;
  if (a.ctrl && !a.ctrl->active) return;
  const int tid = threadIdx.x;
  const int z = blockIdx.y;
  const int y0 = blockIdx.x * C;
  const int ny = a.ny;
  load_twiddles<T, P, NT>(tw, twg, tid);
  for (int e = tid; e < C * KXN; e += NT) {
    const int kx = e / C, col = e % C;
    const int y = y0 + col;
    c4<T> v;
    if (y < ny) v = W2[((size_t)kx * a.nz + z) * ny + y];
    else { v.x = v.y = v.z = v.w = (T)0; }
    // Z(kx) = U + iR
    lds[kx * LD + col] = mk<T>(v.x - v.w, v.y + v.z);
    if (kx > 0 && kx < P / 2) lds[(P - kx) * LD + col] = mk<T>(v.x + v.w, v.z - v.y);
  }
  __syncthreads();
  tile_fft<T, P, C, LD, NT, true, +1>(lds, tw, tid);
  const T sc = (T)a.scale;
  double zz = 0.0, rr = 0.0;
  T* dst = out + ((size_t)z * ny + y0) * NOUT;
  const int rows = min(C, ny - y0);
  for (int e = tid; e < rows * NOUT; e += NT) {
    const int col = e / NOUT, x = e % NOUT;
    const c2<T> v = lds[x * LD + col];
    const T zeta = v.x * sc, res = v.y * sc;
    dst[e] = zeta;
    zz += (double)zeta * zeta;
    rr += (double)res * res;
  }
  if constexpr (MODE == 0) {
    const int nblk = gridDim.x * gridDim.y;
    const int bid = blockIdx.y * gridDim.x + blockIdx.x;
    const double sz = block_sum<NT>(zz, red);
    const double sr = block_sum<NT>(rr, red);
    if (tid == 0) {
      a.norm_part[bid] = make_double2(sr, sz);
      __threadfence();
      last = (atomicAdd(a.ticket, 1u) == (unsigned)(nblk - 1));
    }
    __syncthreads();
    if (!last) return;
    __threadfence();
    double pr = 0.0, pz = 0.0;
    for (int k = tid; k < nblk; k += NT) {
      pr += __hip_atomic_load(&a.norm_part[k].x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      pz += __hip_atomic_load(&a.norm_part[k].y, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const double tr = block_sum<NT>(pr, red);
    const double tz = block_sum<NT>(pz, red);
    if (tid == 0) {
      *a.ticket = 0u;
      ctrl_advance(a.ctrl, tr, tz);
    }
  }
}

// ============================================================ dispatch
#define FR3D_SIZES(X) X(4) X(6) X(8) X(12) X(16) X(24) X(32) X(48) X(64) X(96) X(128) X(192) X(256) X(384) X(512)

inline bool supported_length_impl(int P) {
  switch (P) {
#define X(p) case p:
    FR3D_SIZES(X)
#undef X
    return true;
    default:
      return false;
  }
}

static inline unsigned cdiv(long long a, long long b) { return (unsigned)((a + b - 1) / b); }

template <typename T>
hipError_t launch_fx(int P, bool gen, const T* F, c2<T>* A, const FwdArgs& a, const c2<T>* tw, hipStream_t s) {
  switch (P) {
#define X(p)                                                                                   \
  case p: {                                                                                    \
    dim3 g(cdiv(a.ny_in, 2 * Tile<T, p>::C), a.nz_in);                                         \
    if (gen) hipLaunchKernelGGL((k_fx<T, p, true>), g, dim3(NT), 0, s, F, A, a, tw);           \
    else hipLaunchKernelGGL((k_fx<T, p, false>), g, dim3(NT), 0, s, F, A, a, tw);              \
    break;                                                                                     \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fy(int P, bool prune, const c2<T>* A, c2<T>* B, const FwdArgs& a, const c2<T>* tw, hipStream_t s) {
  const long long nrows = (long long)a.kx_n * a.nz_in;
  switch (P) {
#define X(p)                                                                                   \
  case p: {                                                                                    \
    dim3 g(cdiv(nrows, Tile<T, p>::C));                                                        \
    if (prune) hipLaunchKernelGGL((k_fy<T, p, true>), g, dim3(NT), 0, s, A, B, a, tw);         \
    else hipLaunchKernelGGL((k_fy<T, p, false>), g, dim3(NT), 0, s, A, B, a, tw);              \
    break;                                                                                     \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_fz(int P, int mode, const c2<T>* B, c2<T>* S, const FwdArgs& a, const c2<T>* tw, hipStream_t s) {
  switch (P) {
#define X(p)                                                                                   \
  case p: {                                                                                    \
    const int cols = mode == 0 ? a.py : a.py / 2 + 1;                                          \
    dim3 g(cdiv(cols, Tile<T, p>::C), a.kx_n);                                                 \
    if (mode == 0) hipLaunchKernelGGL((k_fz<T, p, 0>), g, dim3(NT), 0, s, B, S, a, tw);        \
    else hipLaunchKernelGGL((k_fz<T, p, 1>), g, dim3(NT), 0, s, B, S, a, tw);                  \
    break;                                                                                     \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T> constexpr int half_tile(int c) { return c / 2 > 0 ? c / 2 : 1; }

template <typename T>
hipError_t launch_iz(int P, int mode, const c2<T>* S, c4<T>* W1, const InvArgs& a, const c2<T>* tw, hipStream_t s) {
  switch (P) {
#define X(p)                                                                                   \
  case p: {                                                                                    \
    dim3 g(cdiv(a.py, half_tile<T>(Tile<T, p>::C)), a.kx_n);                                   \
    if (mode == 0) hipLaunchKernelGGL((k_iz<T, p, 0>), g, dim3(NT), 0, s, S, W1, a, tw);       \
    else hipLaunchKernelGGL((k_iz<T, p, 1>), g, dim3(NT), 0, s, S, W1, a, tw);                 \
    break;                                                                                     \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_iy(int P, const c4<T>* W1, c4<T>* W2, const InvArgs& a, const c2<T>* tw, hipStream_t s) {
  const long long nrows = (long long)a.kx_n * a.nz;
  switch (P) {
#define X(p)                                                                                   \
  case p: {                                                                                    \
    dim3 g(cdiv(nrows, half_tile<T>(Tile<T, p>::C)));                                          \
    hipLaunchKernelGGL((k_iy<T, p>), g, dim3(NT), 0, s, W1, W2, a, tw);                        \
    break;                                                                                     \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_ix(int P, int mode, const c4<T>* W2, T* out, const InvArgs& a, const c2<T>* tw, hipStream_t s) {
  switch (P) {
#define X(p)                                                                                   \
  case p: {                                                                                    \
    dim3 g(cdiv(a.ny, Tile<T, p>::C), a.nz);                                                   \
    if (mode == 0) hipLaunchKernelGGL((k_ix<T, p, 0>), g, dim3(NT), 0, s, W2, out, a, tw);     \
    else hipLaunchKernelGGL((k_ix<T, p, 1>), g, dim3(NT), 0, s, W2, out, a, tw);               \
    break;                                                                                     \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

#define FR3D_INST(T)                                                                                          \
  template hipError_t launch_fx<T>(int, bool, const T*, c2<T>*, const FwdArgs&, const c2<T>*, hipStream_t);   \
  template hipError_t launch_fy<T>(int, bool, const c2<T>*, c2<T>*, const FwdArgs&, const c2<T>*, hipStream_t); \
  template hipError_t launch_fz<T>(int, int, const c2<T>*, c2<T>*, const FwdArgs&, const c2<T>*, hipStream_t);  \
  template hipError_t launch_iz<T>(int, int, const c2<T>*, c4<T>*, const InvArgs&, const c2<T>*, hipStream_t);  \
  template hipError_t launch_iy<T>(int, const c4<T>*, c4<T>*, const InvArgs&, const c2<T>*, hipStream_t);       \
  template hipError_t launch_ix<T>(int, int, const c4<T>*, T*, const InvArgs&, const c2<T>*, hipStream_t);

}  // namespace fr3d
