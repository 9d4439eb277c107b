// Pass kernels of the padded 3D transforms (layouts in passes.hpp).  Included
// by one translation unit per precision, which instantiates the launchers.
//
// Every kernel first issues all of its global loads into registers, then
// writes the tile to LDS, so each wave keeps its whole share of the tile in
// flight at once; stores go straight from LDS to memory.
#pragma once
#include <hip/hip_ext.h>

#include <type_traits>

#include "passes.hpp"

namespace fr3d {

template <int TOTAL> struct Per {
  static constexpr int n = (TOTAL + NT - 1) / NT;  // elements per thread
  static __device__ __forceinline__ bool ok(int e) { return TOTAL % NT == 0 || e < TOTAL; }
};

// ============================================================ forward x pass
// Real-to-complex transform along x.  Two real rows share one complex pencil
// (a + i b); after the transform A(k) = (Z(k) + conj Z(P-k))/2 and
// B(k) = (Z(k) - conj Z(P-k))/(2i).  Data mode reads the n = P/2 valid
// samples of each row; generator mode samples the kernel's offset table on
// the fly (Sec. 3 kernel, Sec. 5 midpoint weight = cell volume h^2 hz; the
// slot at offset index n is zero).
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

template <typename T, int P, bool GEN, int SHV>
__global__ __launch_bounds__(NT) void k_fx(const T* __restrict__ F, c2<T>* __restrict__ A, FwdArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int SH = SHV & 3, PV = SHV >> 2;  // tile shift, radix plan variant
  constexpr int C = TileC<T, P, SH>::C;  // complex pencils per tile = C, real rows = 2C
  constexpr int LD = RowLD<P>::value;
  constexpr int N = P / 2;
  __shared__ c2<T> lds[C * LD];
  __shared__ c2<T> tw[P];
  const int tid = threadIdx.x;
  const int z = blockIdx.y;
  const int y0 = blockIdx.x * (2 * C);
  const c2<T> twv = twg[tid % P];
  T* ldsr = reinterpret_cast<T*>(lds);
  if constexpr (!GEN) {
    // rows y0 .. y0+2C-1 of plane z are contiguous: 2C*N values
    constexpr int TOT = 2 * C * N;
    using PE = Per<TOT>;
    const int rows = min(2 * C, a.ny_in - y0);
    const T* src = F + ((size_t)z * a.ny_in + y0) * N;
    T v[PE::n];
#pragma unroll
    for (int i = 0; i < PE::n; ++i) {
      const int e = tid + i * NT;
      v[i] = (PE::ok(e) && e / N < rows) ? src[e] : (T)0;
    }
    if (tid < P) tw[tid] = twv;
#pragma unroll
    for (int i = 0; i < PE::n; ++i) {
      const int e = tid + i * NT;
      if (PE::ok(e)) {
        const int r = e / N, x = e % N;
        ldsr[2 * ((r >> 1) * LD + rsw(x)) + (r & 1)] = v[i];
      }
    }
    for (int e = tid; e < C * (P - N); e += NT) {
      const int c = e / (P - N), x = N + e % (P - N);
      lds[c * LD + rsw(x)] = mk<T>(0, 0);
    }
  } else {
    if (tid < P) tw[tid] = twv;
    for (int e = tid; e < 2 * C * P; e += NT) {
      const int r = e / P, x = e % P;
      const int yb = y0 + r;
      double v = 0.0;
      int ox, oy, oz;
      if (a.ksrc) {
        if (yb < a.ny_in) v = a.ksrc[((size_t)z * a.py + yb) * P + x];
      } else {
        const bool zok = a.zlin ? (oz = z - (a.nz - 1), true) : wrap_offset(z, a.nz, a.pz, oz);
        if (yb < a.ny_in && wrap_offset(x, a.nx, P, ox) && wrap_offset(yb, a.ny, a.py, oy) && zok) {
          v = a.h * a.h * a.hz * kernel_value(a.kind, ox * a.h, oy * a.h, (a.D + oz) * a.hz);
        }
      }
      ldsr[2 * ((r >> 1) * LD + rsw(x)) + (r & 1)] = (T)v;
    }
  }
  for (int m = tid + NT; m < P; m += NT) tw[m] = twg[m];
  __syncthreads();
  tile_fft<T, P, C, LD, NT, false, -1, PV>(lds, tw, tid);
  const int kxn = P / 2 + 1;
  for (int e = tid; e < kxn * 2 * C; e += NT) {
    const int yl = e % (2 * C), kx = e / (2 * C);
    const int y = y0 + yl;
    if (y >= a.ny_in) continue;
    const int c = yl >> 1;
    const c2<T> Z = lds[c * LD + rsw(kx)];
    const c2<T> Zm = lds[c * LD + rsw((P - kx) % P)];
    c2<T> v;
    if ((yl & 1) == 0) v = mk<T>((T)0.5 * (Z.x + Zm.x), (T)0.5 * (Z.y - Zm.y));
    else v = mk<T>((T)0.5 * (Z.y + Zm.y), (T)0.5 * (Zm.x - Z.x));
    A[((size_t)kx * a.nz_in + z) * a.ny_in + y] = v;
  }
}

// ============================================================ forward y pass
// Complex transform along y of every row (kx, z); rows are contiguous.
template <typename T, int P, bool PRUNE, int SHV>
__global__ __launch_bounds__(NT) void k_fy(const c2<T>* __restrict__ A, c2<T>* __restrict__ B, FwdArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int SH = SHV & 3, PV = SHV >> 2;  // tile shift, radix plan variant
  constexpr int C = TileC<T, P, SH>::C;
  constexpr int LD = RowLD<P>::value;
  constexpr int NIN = PRUNE ? P / 2 : P;
  constexpr int TOT = C * NIN;
  using PE = Per<TOT>;
  __shared__ c2<T> lds[C * LD];
  __shared__ c2<T> tw[P];
  const int tid = threadIdx.x;
  const long long nrows = (long long)a.kx_n * a.nz_in;
  const long long row0 = (long long)blockIdx.x * C;
  const int rows = (int)min((long long)C, nrows - row0);
  const c2<T>* src = A + row0 * NIN;
  c2<T> v[PE::n];
#pragma unroll
  for (int i = 0; i < PE::n; ++i) {
    const int e = tid + i * NT;
    v[i] = (PE::ok(e) && e / NIN < rows) ? src[e] : mk<T>(0, 0);
  }
  for (int m = tid; m < P; m += NT) tw[m] = twg[m];
#pragma unroll
  for (int i = 0; i < PE::n; ++i) {
    const int e = tid + i * NT;
    if (PE::ok(e)) lds[(e / NIN) * LD + rsw(e % NIN)] = v[i];
  }
  if constexpr (PRUNE) {
    for (int e = tid; e < C * (P - NIN); e += NT) {
      const int r = e / (P - NIN), y = NIN + e % (P - NIN);
      lds[r * LD + rsw(y)] = mk<T>(0, 0);
    }
  }
  __syncthreads();
  tile_fft<T, P, C, LD, NT, false, -1, PV>(lds, tw, tid);
  c2<T>* dst = B + row0 * P;
  for (int e = tid; e < rows * P; e += NT) dst[e] = lds[(e / P) * LD + rsw(e % P)];
}

// ============================================================ forward z pass
// Complex transform along z of C consecutive ky-columns of one kx plane.
// MODE 0 (data): n inputs, P outputs, fused energy epilogue writing
// per-workgroup partials of the energy per kernel-spectrum level.  MODE 1 (kernel spectrum): P inputs, only
// kz <= P/2 and ky <= Py/2 stored (the octant).
// Slot of a forward z workgroup's bin partials (the grid is a multiple of
// 8 workgroups): workgroups of one XCD (w mod 8) fill adjacent slots, so each
// 128 B line of a bin's row of partials is written from one XCD's L2.
__device__ __forceinline__ int bins_slot(int w, int nblk) { return (w & 7) * (nblk >> 3) + (w >> 3); }

template <typename T, int P, int MODE, int SHV>
__global__ __launch_bounds__(NT) void k_fz(const c2<T>* __restrict__ B, c2<T>* __restrict__ S, FwdArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int SH = SHV & 3, PV = SHV >> 2;  // tile shift, radix plan variant
  constexpr int C = TileC<T, P, SH>::C;
  constexpr int LD = C;
  constexpr int NIN = MODE == 0 ? P / 2 : P;
  constexpr int NOUT = MODE == 0 ? P : P / 2 + 1;
  constexpr int TOT = C * NIN;
  using PE = Per<TOT>;
  __shared__ c2<T> lds[P * LD];
  __shared__ c2<T> tw[P];
  // two copies of the 64 feature bins, for even and odd lanes: neighbouring
  // lanes (neighbouring ky columns) mostly hit the same level, and their
  // LDS atomics on one address serialise
  __shared__ double bins2[2 * 64];
  double* bins = bins2 + 64 * (threadIdx.x & 1);
  const int tid = threadIdx.x;
  const int py = a.py;
  int kx, tile;
  if constexpr (MODE == 0) {
    // tiles 2t and 2t+1 share the 128 B lines of B's rows: they run as
    // workgroups w and w + 8, i.e. on the same XCD (round robin over 8), so
    // the second read of a line hits that XCD's L2
    const int ntile = (py + C - 1) / C, npr = (ntile + 1) / 2;
    const int w = blockIdx.x, sidx = w >> 3;
    const int pidx = (sidx >> 1) * 8 + (w & 7);
    kx = pidx / npr;
    tile = 2 * (pidx % npr) + (sidx & 1);
    if (kx >= a.kx_n || tile >= ntile) {  // padding of the grid: an empty partial
      if (tid < 64) a.bins_part[(size_t)tid * gridDim.x + bins_slot(blockIdx.x, gridDim.x)] = 0.0;
      return;
    }
  } else {
    kx = blockIdx.y;
    tile = blockIdx.x;
  }
  const int ky0 = tile * C;
  const c2<T>* src = B + (size_t)kx * NIN * py;
  c2<T> v[PE::n];
#pragma unroll
  for (int i = 0; i < PE::n; ++i) {
    const int e = tid + i * NT;
    const int ky = ky0 + e % C;
    v[i] = (PE::ok(e) && ky < py) ? src[(size_t)(e / C) * py + ky] : mk<T>(0, 0);
  }
  // data mode, run layout (each thread one column's run of RPC consecutive
  // kz): the feature levels of the run, loaded with the data so that their
  // latency hides behind the transform, four per word
  constexpr bool RUN = C <= NT && NT % C == 0 && (C * P / NT) % 4 == 0;
  constexpr int RPC = RUN ? C * P / NT : 4;
  uint32_t lvw[RPC / 4] = {};
  if constexpr (MODE == 0 && RUN) {
    const int ky = ky0 + tid % C, k0 = (tid / C) * RPC;
    if (ky < py) {
      // the table row of (kx, |ky|) over all kz: RPC consecutive bytes from k0
      const uint32_t* lrow = reinterpret_cast<const uint32_t*>(
          a.level + ((size_t)kx * (py / 2 + 1) + (ky <= py / 2 ? ky : py - ky)) * P + k0);
#pragma unroll
      for (int j = 0; j < RPC / 4; ++j) lvw[j] = lrow[j];
    }
  }
  for (int m = tid; m < P; m += NT) tw[m] = twg[m];
  if (MODE == 0 && tid < 2 * 64) bins2[tid] = 0.0;
#pragma unroll
  for (int i = 0; i < PE::n; ++i) {
    const int e = tid + i * NT;
    if (PE::ok(e)) lds[e] = v[i];  // row e / C, column e % C
  }
  if constexpr (NIN < P) {
    for (int e = tid; e < C * (P - NIN); e += NT) lds[NIN * LD + e] = mk<T>(0, 0);
  }
  __syncthreads();
  tile_fft<T, P, C, LD, NT, true, -1, PV>(lds, tw, tid);
  if constexpr (MODE == 0) {
    const int lg = spec_lg(sizeof(T), P, py);
    c2<T>* dst = S + (size_t)kx * spec_plane(P, py, lg);
    const double w = (kx == 0 || 2 * kx == a.bg.px) ? 1.0 : 2.0;
    // the kernel-spectrum level of (kx, ky, kz): table row (kx, |ky|), entry kz
    const uint8_t* lev = a.level + (size_t)kx * (py / 2 + 1) * P;
    // the tile's C columns are C / G whole granules, consecutive in S: one
    // contiguous range, written in storage order (columns past Py skipped)
    {
      c2<T>* out = dst + (((size_t)(ky0 >> lg) * P) << lg);
      const int gm = (1 << lg) - 1;
#pragma unroll
      for (int i = 0; i < (C * P + NT - 1) / NT; ++i) {
        const int e = tid + i * NT;
        if ((C * P) % NT != 0 && e >= C * P) break;
        const int r = e >> lg, kz = r % P, col = ((r / P) << lg) + (e & gm);
        if (ky0 + col < py) out[e] = lds[kz * LD + col];
      }
    }
    int cur = -1;
    double acc = 0.0;
    auto visit = [&](int kz, int col) {
      const int ky = ky0 + col;
      if (ky >= py) return;
      const c2<T> u = lds[kz * LD + col];
      const int my = ky <= py / 2 ? ky : py - ky;
      const int b = lev[(size_t)my * P + kz];
      if (b != cur) {
        if (cur >= 0) atomicAdd(&bins[cur], acc);
        cur = b;
        acc = 0.0;
      }
      acc += w * ((double)u.x * u.x + (double)u.y * u.y);
    };
    // energies: a second read of the tile
    if constexpr (RUN) {
      // each thread walks a run of consecutive kz in one column, so its bin
      // changes rarely and few LDS atomics are needed
      const int col = tid % C, k0 = (tid / C) * RPC;
      const int ky = ky0 + col;
      if (ky < py) {
#pragma unroll
        for (int j = 0; j < RPC; ++j) {
          const int kz = k0 + j;
          const c2<T> u = lds[kz * LD + col];
          const int b = (int)((lvw[j >> 2] >> (8 * (j & 3))) & 255u);
          if (b != cur) {
            if (cur >= 0) atomicAdd(&bins[cur], acc);
            cur = b;
            acc = 0.0;
          }
          acc += w * ((double)u.x * u.x + (double)u.y * u.y);
        }
      }
    } else {
      for (int e = tid; e < C * P; e += NT) visit(e / C, e % C);
    }
    if (cur >= 0) atomicAdd(&bins[cur], acc);
    __syncthreads();
    const int bid = blockIdx.x, nblk = gridDim.x;
    if (tid < 64) a.bins_part[(size_t)tid * nblk + bins_slot(bid, nblk)] = bins2[tid] + bins2[64 + tid];
  } else {
    const int oy = py / 2 + 1;
    c2<T>* dst = S + (size_t)kx * NOUT * oy;
    for (int e = tid; e < C * NOUT; e += NT) {
      const int kz = e / C, col = e % C;
      const int ky = ky0 + col;
      if (ky < oy) dst[(size_t)kz * oy + ky] = lds[e];
    }
  }
}

// ============================================================ inverse z pass
// Reads f^ for C ky-columns of one kx plane and all kz, forms per point (the
// coefficients in T's precision from the FP64 octant of k^):
//   MODE 0: u^ = conj(k^) f^ g(s),  r^ = -e(s) f^   with s = |k^|^2 and the
//           regularising filter (Sec. 4-5):
//             Tikhonov           g = 1/(s + a),                 e = a/(s + a)
//             iterated, order m  g = sum_{j<m} q^j / (s + a),   e = q^m,  q = a/(s + a)
//             truncated SVD      g = 1/s, e = 0 if s >= a;      g = 0, e = 1 otherwise
//   MODE 1: u^ = k^ f^ (a.adj: conj(k^) f^, the adjoint),  r^ = 0  (forward operator)
// transforms u^ and then r^ along z in the same LDS tile and writes z < nz
// as (u, r) pairs.
//
// 1/x for normal positive x: the hardware estimate refined by two Newton
// steps r <- r + r (1 - x r), within an ulp of the quotient (FP32: one step).
__device__ __forceinline__ double recip(double x) {
  double r = __builtin_amdgcn_rcp(x);
  r = fma(r, fma(-x, r, 1.0), r);
  return fma(r, fma(-x, r, 1.0), r);
}
__device__ __forceinline__ float recipf(float x) {
  const float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}

// Octant reuse: rows kz and P-kz need the same octant entry (conjugated), so
// each thread loads f^ for such a pair of rows and the octant entry once.
// Tiles 2m and 2m + 1 of a plane read neighbouring columns of the octant's
// rows (the same 128 B lines when a tile's row segment is shorter than a
// line) and the mirrored pair (tiles of line pair L - 1 - m) the mirrored
// columns ky -> Py - ky; the four run as workgroups w, w + 8, w + 16, w + 24,
// i.e. on one XCD (workgroups go to the XCDs round robin), so the second
// read of a line or of an octant column hits that XCD's L2.  Each XCD takes
// a contiguous range of these groups in order: the octant line at the edge
// between neighbouring groups (the mirrored columns are offset by one) is
// then read by the same XCD in consecutive groups.
__device__ __forceinline__ bool xcd_quad_map(int w, int nplane, int ntile, int& plane, int& tile) {
  const int L = (ntile + 1) / 2, G = (L + 1) / 2;  // line pairs, groups per plane
  const int ngroups = nplane * G, per = (ngroups + 7) / 8;  // groups per XCD
  const int x = w & 7, s = w >> 3;
  const int sub = s & 3, q = s >> 2;
  if (q >= per) return false;
  const int grp = x * per + q;
  if (grp >= ngroups) return false;
  plane = grp / G;
  const int gi = grp % G;
  const int m2 = L - 1 - gi;
  if (sub >= 2 && m2 == gi) return false;  // the middle line pair is its own mirror
  tile = 2 * (sub < 2 ? gi : m2) + (sub & 1);
  return tile < ntile;
}

// K32: the FP32 Tikhonov-family filter reads the kernel spectrum as FP32
// (a.oct32, the FP64 octant rounded once), the values it rounds to anyway.
template <typename T, int P, int MODE, int SHV, bool KM, bool K32 = false>
__global__ __launch_bounds__(NT) void k_iz(const c2<T>* __restrict__ S, c4<T>* __restrict__ W1, InvArgs a,
                                           const c2<T>* __restrict__ twg) {
  static_assert(!K32 || (sizeof(T) == 4 && MODE == 0), "FP32 spectrum: FP32 filter only");
  using KT = typename std::conditional<K32, float2, double2>::type;
  constexpr int SH = SHV & 3, PV = SHV >> 2;  // tile shift, radix plan variant
  // SH = 2 (joint variant, Tikhonov mode): C ky columns of the half tile, u^
  // and r^ side by side as 2C pencils, transformed together.
  constexpr bool JOINT = SH == 2 && MODE == 0;
  constexpr int C = TileC<T, P, JOINT ? 1 : SH>::C;
  constexpr int LD = JOINT ? 2 * C : C;
  constexpr int NOUT = P / 2;
  constexpr int TOT = C * P;
  constexpr int TOTO = C * NOUT;
  using PE = Per<TOT>;
  using PO = Per<TOTO>;
  constexpr bool PAIRED = C <= NT && NT % C == 0 && (P / 2) % (NT / C) == 0;
  __shared__ c2<T> lds[P * LD];
  __shared__ c2<T> tw[P];
  double alpha1;  // the single evaluation's alpha
  if (inv_idle(a, alpha1)) return;
  // candidates [cb, ce) of a K-candidate step, else the single evaluation
  int cb = 0, ce = 1;
  if constexpr (KM) {
    cb = blockIdx.y * a.kb;
    ce = min(cb + a.kb, a.ctrl->kc);
    if (cb >= ce) return;
    W1 = (c4<T>*)a.ctrl->kw1;  // the search's K-candidate workspace
  }
  const int py = a.py;
  const int ntile = (py + C - 1) / C;
  int kx, tile;
  const bool mine = xcd_quad_map(blockIdx.x, a.kx_n, ntile, kx, tile);
  if (!mine) return;
  const int tid = threadIdx.x;
  const int ky0 = tile * C;
  const int oz = P / 2 + 1, oy = py / 2 + 1;
  const int lg = spec_lg(sizeof(T), P, py);
  const c2<T>* src = S + (size_t)kx * spec_plane(P, py, lg);
  const KT* oc;
  if constexpr (K32) oc = a.oct32 + (size_t)kx * oz * oy;
  else oc = a.oct + (size_t)kx * oz * oy;
  // filter of one point: u and r from f^ and the (possibly conjugated) k^;
  // returns the residual factor (r^ = cr f^; 0 for the forward operator)
  auto filt = [&](double aa, c2<T> f, KT kk, c2<T>& u, c2<T>& r) -> T {
    const double fx = (double)f.x, fy = (double)f.y;
    if constexpr (MODE == 0 && sizeof(T) == 4) {
      // FP32 transforms filter in FP32: the coefficients from the FP64
      // spectrum rounded to FP32 (relative error ~1e-7, the order of the
      // transforms' own rounding); the TSVD cut is decided in FP64
      const float kxf = (float)kk.x, kyf = (float)kk.y, aaf = (float)aa;
      const float sf = fmaf(kxf, kxf, kyf * kyf);
      float gu, cr;
      if (a.filt == 0) {
        gu = recipf(sf + aaf);
        cr = -aaf * gu;
      } else if (a.filt == 1) {
        const float d = recipf(sf + aaf), q = aaf * d;
        float qp = 1.0f, sum = 1.0f;
        for (int j = 1; j < a.order; ++j) {
          qp *= q;
          sum += qp;
        }
        gu = d * sum;
        cr = -(qp * q);
      } else {
        const bool keep = kk.x * kk.x + kk.y * kk.y >= aa;
        gu = keep ? recipf(sf) : 0.0f;
        cr = keep ? 0.0f : -1.0f;
      }
      const float cx = kxf * gu, cy = -kyf * gu;  // conj(k^) g
      u = mk<T>((T)(f.x * cx - f.y * cy), (T)(f.x * cy + f.y * cx));
      r = mk<T>((T)(f.x * cr), (T)(f.y * cr));
      return (T)cr;
    } else if constexpr (MODE == 0) {
      const double s = kk.x * kk.x + kk.y * kk.y;
      double gu, cr;
      if (a.filt == 0) {
        gu = recip(s + aa);
        cr = -aa * gu;
      } else if (a.filt == 1) {
        const double d = recip(s + aa), q = aa * d;
        double qp = 1.0, sum = 1.0;
        for (int j = 1; j < a.order; ++j) {
          qp *= q;
          sum += qp;
        }
        gu = d * sum;
        cr = -(qp * q);
      } else {
        const bool keep = s >= aa;
        gu = keep ? recip(s) : 0.0;
        cr = keep ? 0.0 : -1.0;
      }
      const double cx = kk.x * gu, cy = -kk.y * gu;  // conj(k^) g
      u = mk<T>((T)(fx * cx - fy * cy), (T)(fx * cy + fy * cx));
      r = mk<T>((T)(fx * cr), (T)(fy * cr));
      return (T)cr;
    } else {
      const double kyv = a.adj ? -kk.y : kk.y;  // adjoint: conj(k^), the correlation with K
      u = mk<T>((T)(fx * kk.x - fy * kyv), (T)(fx * kyv + fy * kk.x));
      r = mk<T>(0, 0);
      return (T)0;
    }
  };
  // Tikhonov residual r^ = -e f^ with e = a / (s + a) = -cr: ||r||^2 sums
  // w e^2 |f^|^2 and its derivative in ln a sums 2 w e^2 (1 - e) |f^|^2.
  // Summed on every evaluation (a few FMAs; a branch here would split the
  // unrolled filter loop), reduced only when the slope is wanted.
  T sa = 0, sb = 0;
  auto slope_add = [&](c2<T> r, T cr) {
    const T q = r.x * r.x + r.y * r.y;
    sa += q;
    sb += q * (1 + cr);
  };
  // loads: kept in registers across the candidates
  constexpr int TPC = PAIRED ? NT / C : 1;         // threads per column
  constexpr int UPT = PAIRED ? (P / 2) / TPC : 1;  // row pairs per thread
  constexpr int NF = PAIRED ? UPT : PE::n;
  c2<T> f0[NF], f1[PAIRED ? UPT : 1];
  const KT k0{0, 0};
  KT k[NF];
  KT kmid = k0;
  if constexpr (PAIRED) {
    const int col = tid % C, j = tid / C;
    const int ky = ky0 + col;
    const bool okc = ky < py;
    const int my = ky <= py / 2 ? ky : py - ky;
#pragma unroll
    for (int i = 0; i < UPT; ++i) {
      const int p = j + TPC * i;  // rows p and P-p (p = 0: rows 0 and P/2)
      const int r1 = p == 0 ? P / 2 : P - p;
      f0[i] = okc ? src[spec_off(p, ky, P, lg)] : mk<T>(0, 0);
      f1[i] = okc ? src[spec_off(r1, ky, P, lg)] : mk<T>(0, 0);
      k[i] = okc ? oc[(size_t)p * oy + my] : k0;
    }
    if (j == 0 && okc) kmid = oc[(size_t)(P / 2) * oy + my];
  } else {
#pragma unroll
    for (int i = 0; i < PE::n; ++i) {
      const int e = tid + i * NT;
      const int kz = e / C, ky = ky0 + e % C;
      const bool ok = PE::ok(e) && ky < py;
      const int mz = kz <= P / 2 ? kz : P - kz;
      const int my = ky <= py / 2 ? ky : py - ky;
      f0[i] = ok ? src[spec_off(kz, ky, P, lg)] : mk<T>(0, 0);
      k[i] = ok ? oc[(size_t)mz * oy + my] : k0;
    }
  }
  for (int m = tid; m < P; m += NT) tw[m] = twg[m];
  for (int cand = cb; cand < ce; ++cand) {
    const double aa = MODE == 0 ? (KM ? a.ctrl->ca[cand] : alpha1) : 0.0;
    if (KM && cand > cb) __syncthreads();  // the previous candidate's stores have read the tile
    c2<T> r[PE::n];
    if constexpr (PAIRED) {
      const int col = tid % C, j = tid / C;
#pragma unroll
      for (int i = 0; i < UPT; ++i) {
        const int p = j + TPC * i;
        const int r1 = p == 0 ? P / 2 : P - p;
        c2<T> u0, u1;
        const T c0 = filt(aa, f0[i], k[i], u0, r[2 * i]);
        KT k1 = k[i];
        if (p == 0) k1 = kmid;
        else k1.y = -k1.y;  // row P-p > P/2: conj
        const T c1 = filt(aa, f1[i], k1, u1, r[2 * i + 1]);
        slope_add(r[2 * i], c0);
        slope_add(r[2 * i + 1], c1);
        lds[p * LD + col] = u0;
        lds[r1 * LD + col] = u1;
        if constexpr (JOINT) {
          lds[p * LD + C + col] = r[2 * i];
          lds[r1 * LD + C + col] = r[2 * i + 1];
        }
      }
    } else {
#pragma unroll
      for (int i = 0; i < PE::n; ++i) {
        const int e = tid + i * NT;
        KT kk = k[i];
        if (e / C > P / 2) kk.y = -kk.y;
        c2<T> u;
        const T c0 = filt(aa, f0[i], kk, u, r[i]);
        slope_add(r[i], c0);
        if (PE::ok(e)) {
          lds[(e / C) * LD + e % C] = u;
          if constexpr (JOINT) lds[(e / C) * LD + C + e % C] = r[i];
        }
      }
    }
    if constexpr (MODE == 0 && !KM) {
      // the seed of a secant search with a slope ratio (the host passes
      // slope_part for that launch only): each wave's partials, with the
      // half-spectrum weight w (no LDS)
      if (a.slope_part && a.filt == 0) {
        const double w = (kx == 0 || kx == a.kx_n - 1) ? 1.0 : 2.0;
        const double A = wave_sum<double>((double)sa);
        const double B = wave_sum<double>((double)sb);
        if ((tid & 63) == 0) a.slope_part[(size_t)blockIdx.x * (NT / 64) + (tid >> 6)] = make_double2(w * A, w * B);
      }
    }
    __syncthreads();
    if constexpr (JOINT) {
      tile_fft<T, P, 2 * C, LD, NT, true, +1, PV>(lds, tw, tid);
      c4<T>* dst = W1 + (KM ? (size_t)cand * a.w1_stride : 0) + (size_t)kx * NOUT * py;
#pragma unroll
      for (int i = 0; i < PO::n; ++i) {
        const int e = tid + i * NT;
        const int z = e / C, col = e % C, ky = ky0 + col;
        if (!PO::ok(e) || ky >= py) continue;
        const c2<T> u = lds[z * LD + col], w = lds[z * LD + C + col];
        c4<T> v;
        v.x = u.x; v.y = u.y; v.z = w.x; v.w = w.y;
        dst[(size_t)z * py + ky] = v;
      }
      continue;
    }
    tile_fft<T, P, C, LD, NT, true, +1, PV>(lds, tw, tid);
    c2<T> uo[PO::n];
#pragma unroll
    for (int i = 0; i < PO::n; ++i) {
      const int e = tid + i * NT;
      uo[i] = PO::ok(e) ? lds[e] : mk<T>(0, 0);
    }
    __syncthreads();
    if constexpr (PAIRED) {
      const int col = tid % C, j = tid / C;
#pragma unroll
      for (int i = 0; i < UPT; ++i) {
        const int p = j + TPC * i;
        const int r1 = p == 0 ? P / 2 : P - p;
        lds[p * LD + col] = r[2 * i];
        lds[r1 * LD + col] = r[2 * i + 1];
      }
    } else {
#pragma unroll
      for (int i = 0; i < PE::n; ++i) {
        const int e = tid + i * NT;
        if (PE::ok(e)) lds[e] = r[i];
      }
    }
    __syncthreads();
    if constexpr (MODE == 0) tile_fft<T, P, C, LD, NT, true, +1, PV>(lds, tw, tid);
    c4<T>* dst = W1 + (KM ? (size_t)cand * a.w1_stride : 0) + (size_t)kx * NOUT * py;
#pragma unroll
    for (int i = 0; i < PO::n; ++i) {
      const int e = tid + i * NT;
      const int z = e / C, ky = ky0 + e % C;
      if (!PO::ok(e) || ky >= py) continue;
      const c2<T> w = lds[e];
      c4<T> v;
      v.x = uo[i].x; v.y = uo[i].y; v.z = w.x; v.w = w.y;
      dst[(size_t)z * py + ky] = v;
    }
  }
}

// ============================================================ inverse y pass
// Rows (kx, z) of (u, r) pairs: both transformed along y, y < ny written.
template <typename T, int P, int SHV>
__global__ __launch_bounds__(NT) void k_iy(const c4<T>* __restrict__ W1, c4<T>* __restrict__ W2, InvArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int SH = SHV & 3, PV = SHV >> 2;  // tile shift, radix plan variant
  constexpr int C = TileC<T, P, SH + 1>::C;  // rows per tile (two pencils each)
  constexpr int NC = 2 * C;
  constexpr int LD = RowLD<P>::value;
  constexpr int NOUT = P / 2;
  constexpr int TOT = C * P;
  using PE = Per<TOT>;
  __shared__ c2<T> lds[NC * LD];
  __shared__ c2<T> tw[P];
  if (inv_idle(a)) return;
  const int cand = a.kmode ? (int)blockIdx.y : 0;  // candidate of a K-candidate step
  if (a.kmode) {
    if (cand >= a.ctrl->kc) return;
    W1 = (const c4<T>*)a.ctrl->kw1 + (size_t)cand * a.w1_stride;
    W2 = (c4<T>*)a.ctrl->kw2 + (size_t)cand * a.w2_stride;
  }
  const int tid = threadIdx.x;
  const long long nrows = (long long)a.kx_n * a.nz;
  const long long row0 = (long long)blockIdx.x * C;
  const int rows = (int)min((long long)C, nrows - row0);
  const c4<T>* src = W1 + row0 * P;
  c4<T> v[PE::n];
#pragma unroll
  for (int i = 0; i < PE::n; ++i) {
    const int e = tid + i * NT;
    if (PE::ok(e) && e / P < rows) v[i] = src[e];
    else { v[i].x = v[i].y = v[i].z = v[i].w = (T)0; }
  }
  for (int m = tid; m < P; m += NT) tw[m] = twg[m];
#pragma unroll
  for (int i = 0; i < PE::n; ++i) {
    const int e = tid + i * NT;
    if (!PE::ok(e)) continue;
    const int r = e / P, y = e % P;
    lds[(2 * r) * LD + rsw(y)] = mk<T>(v[i].x, v[i].y);
    lds[(2 * r + 1) * LD + rsw(y)] = mk<T>(v[i].z, v[i].w);
  }
  __syncthreads();
  tile_fft<T, P, NC, LD, NT, false, +1, PV>(lds, tw, tid);
  c4<T>* dst = W2 + row0 * NOUT;
  for (int e = tid; e < rows * NOUT; e += NT) {
    const int r = e / NOUT, y = e % NOUT;
    const c2<T> u = lds[(2 * r) * LD + rsw(y)], w = lds[(2 * r + 1) * LD + rsw(y)];
    c4<T> o;
    o.x = u.x; o.y = u.y; o.z = w.x; o.w = w.y;
    dst[e] = o;
  }
}

// ============================================================ inverse x pass
// For C consecutive y of one z: u and r are Hermitian in kx (their 3D
// transforms are real), so Z(kx) = U(kx) + i R(kx) over the full kx range
// (Z(P-kx) = conj U(kx) + i conj R(kx)) transforms to u + i r.  Writes
// zeta = Re/P^3 on R (MODE 0 and 1) and accumulates ||zeta||^2 and
// ||r||^2 = sum (Im/P^3)^2 in FP64; the last workgroup sums the partials in
// a fixed order and advances the alpha search (MODE 0).
template <typename T, int P, int MODE, int SHV>
__global__ __launch_bounds__(NT) void k_ix(const c4<T>* __restrict__ W2, T* __restrict__ out, InvArgs a,
                                           const c2<T>* __restrict__ twg) {
  constexpr int SH = SHV & 3, PV = SHV >> 2;  // tile shift, radix plan variant
  constexpr int C = TileC<T, P, SH>::C;
  constexpr int LD = C + 1;
  constexpr int NOUT = P / 2;
  constexpr int KXN = P / 2 + 1;
  constexpr int TOT = C * KXN;
  using PE = Per<TOT>;
  __shared__ c2<T> lds[P * LD];
  __shared__ c2<T> tw[P];
  // the norm reduction's scratch lives in the twiddle table, unused after
  // the transform (at 512 points a separate array would cost a workgroup per CU)
  double* red = reinterpret_cast<double*>(tw);
  if (inv_idle(a)) return;
  const int cand = a.kmode ? (int)blockIdx.z : 0;  // candidate of a K-candidate step
  if (a.kmode) {
    if (cand >= a.ctrl->kc) return;
    W2 = (const c4<T>*)a.ctrl->kw2 + (size_t)cand * a.w2_stride;
  }
  const int tid = threadIdx.x;
  const int z = blockIdx.y;
  const int y0 = blockIdx.x * C;
  const int ny = a.ny;
  c4<T> v[PE::n];
#pragma unroll
  for (int i = 0; i < PE::n; ++i) {
    const int e = tid + i * NT;
    const int kx = e / C, y = y0 + e % C;
    if (PE::ok(e) && y < ny) v[i] = W2[((size_t)kx * a.nz + z) * ny + y];
    else { v[i].x = v[i].y = v[i].z = v[i].w = (T)0; }
  }
  for (int m = tid; m < P; m += NT) tw[m] = twg[m];
#pragma unroll
  for (int i = 0; i < PE::n; ++i) {
    const int e = tid + i * NT;
    if (!PE::ok(e)) continue;
    const int kx = e / C, col = e % C;
    // Z(kx) = U + iR
    lds[kx * LD + col] = mk<T>(v[i].x - v[i].w, v[i].y + v[i].z);
    if (kx > 0 && kx < P / 2) lds[(P - kx) * LD + col] = mk<T>(v[i].x + v[i].w, v[i].z - v[i].y);
  }
  __syncthreads();
  tile_fft<T, P, C, LD, NT, true, +1, PV>(lds, tw, tid);
  const T sc = (T)a.scale;
  double zz = 0.0, rr = 0.0;
  if (a.ctrl) out = (T*)a.ctrl->out;  // a search writes the zeta its control block names
  T* dst = out + ((size_t)z * ny + y0) * NOUT;
  const int rows = min(C, ny - y0);
  for (int e = tid; e < rows * NOUT; e += NT) {
    const int col = e / NOUT, x = e % NOUT;
    const c2<T> u = lds[x * LD + col];
    const T zeta = u.x * sc, res = u.y * sc;
    if (!a.kmode) dst[e] = zeta;
    zz += (double)zeta * zeta;
    rr += (double)res * res;
  }
  if constexpr (MODE == 0) {
    const int bid = blockIdx.y * gridDim.x + blockIdx.x;
    const double sz = block_sum<NT>(zz, red);
    const double sr = block_sum<NT>(rr, red);
    if (tid == 0) (a.kmode ? a.ctrl->knorm : a.norm_part)[(size_t)cand * a.norm_stride + bid] = make_double2(sr, sz);
  }
}

// Final sum of the x pass's norm partials in a fixed order (one workgroup),
// then one step of the alpha search.
// With the z pass's slope partials (seed of a secant search), also the
// full-box slope d ln ||r|| / d log10 a = ln 10 sum w e^2 (1 - e) |f^|^2 /
// sum w e^2 |f^|^2.
static __global__ __launch_bounds__(NT) void k_norm_final(InvArgs a, int nblk) {
  __shared__ double red[NT / 64];
  if (inv_idle(a)) return;
  const double2 p = strided_sum<double2>(a.norm_part, threadIdx.x, nblk, NT);
  const double tr = block_sum<NT>(p.x, red);
  const double tz = block_sum<NT>(p.y, red);
  double sfull = -1.0;
  if (a.slope_part && a.filt == 0 && ctrl_wants_slope(a.ctrl)) {
    // the wave entries of workgroups with a tile, each thread over a fixed
    // stride of workgroups
    double2 q = make_double2(0.0, 0.0);
    for (int w = threadIdx.x; w < a.slope_n; w += NT) {
      int kx, tile;
      const bool mine = xcd_quad_map(w, a.kx_n, a.slope_ntile, kx, tile);
      if (mine) {
#pragma unroll
        for (int i = 0; i < NT / 64; ++i) {
          const double2 v = a.slope_part[(size_t)w * (NT / 64) + i];
          q.x += v.x;
          q.y += v.y;
        }
      }
    }
    const double A = block_sum<NT>(q.x, red);
    const double B = block_sum<NT>(q.y, red);
    if (A > 0) sfull = 2.302585092994045684 * B / A;
  }
  if (threadIdx.x == 0) ctrl_advance(a.ctrl, tr, tz, sfull);
}

// The same for the kc candidates of a K-candidate step: wave w sums the
// partials of candidates w, w + 4, ... in a fixed order, then one step of
// the K-candidate search.
static __global__ __launch_bounds__(NT) void k_norm_final_k(InvArgs a, int nblk) {
  __shared__ double r2[KMAX], z2[KMAX];
  if (inv_idle(a)) return;
  const int kc = a.ctrl->kc;
  const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
  for (int j = w; j < kc; j += NT / 64) {
    const double2 p = strided_sum<double2>(a.ctrl->knorm + (size_t)j * a.norm_stride, lane, nblk, 64);
    const double pr = wave_sum<double>(p.x);
    const double pz = wave_sum<double>(p.y);
    if (lane == 0) { r2[j] = pr; z2[j] = pz; }
  }
  __syncthreads();
  if (threadIdx.x == 0) ctrl_advance_k(a.ctrl, r2, z2);
}

// Level energies and predictor features from the z pass's per-workgroup bin
// partials: workgroup b sums bin b over all partials in a fixed order; the
// last workgroup forms x_b = log10(E_b / mean E + 1e-30) and
// x_64 = log10(delta / ||F||) with ||F||^2 = sum E / (Px Py Pz) (Parseval).
static __global__ __launch_bounds__(NT) void k_bins_final(FwdArgs a, int nblk) {
  __shared__ double red[NT / 64];
  __shared__ int last;
  const int b = blockIdx.x;
  const double* row = a.bins_part + (size_t)b * nblk;
  double s = strided_sum<double, 16>(row, threadIdx.x, nblk, NT);
  s = block_sum<NT>(s, red);
  if (threadIdx.x == 0) {
    a.bins_out[b] = s;
    __threadfence();
    last = (atomicAdd(a.ticket, 1u) == 63u);
  }
  __syncthreads();
  if (!last) return;
  __threadfence();
  if (threadIdx.x < 64) {
    const double E = __hip_atomic_load(&a.bins_out[threadIdx.x], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const double tot = wave_sum<double>(E);
    a.feat_out[threadIdx.x] = (float)log10(E / (tot / 64.0) + 1e-30);
    if (threadIdx.x == 0) {
      const double fnorm = sqrt(tot / ((double)a.bg.px * a.bg.py * a.bg.pz));
      a.feat_out[64] = (float)log10(a.delta / fnorm);
      *a.ticket = 0u;
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

template <typename K, typename... Args>
static inline hipError_t go(K kern, dim3 g, const Launch& L, Args... args) {
  if (L.e0) hipExtLaunchKernelGGL(kern, g, dim3(NT), 0, L.s, L.e0, L.e1, 0, args...);
  else hipLaunchKernelGGL(kern, g, dim3(NT), 0, L.s, args...);
  return hipGetLastError();
}

// Compiled variants of a pass kernel: the tile shift (0 = 32 KiB tile, 1 =
// half, 2 = quarter; lengths below 64 only 0) and, for the FP32 transforms of
// lengths 192, 384 and 512, the radix plan variant (0-2), encoded as the
// template argument SHV = shift + 4 variant.  A launch's Launch::sh holds the
// same encoding; `pick` maps it to a compiled instance and calls f with it.
template <int V> using IC = std::integral_constant<int, V>;
template <typename T, int p> constexpr bool plan_variants() { return sizeof(T) == 4 && (p == 192 || p == 384 || p == 512); }

template <int NSH, int V, typename F> static inline hipError_t pick_sh(int sh, F&& f) {
  if constexpr (NSH > 2) {
    if (sh >= 2) return f(IC<2 + 4 * V>{});
  }
  if constexpr (NSH > 1) {
    if (sh >= 1) return f(IC<1 + 4 * V>{});
  }
  return f(IC<4 * V>{});
}

// NSH: the tile shifts the pass has (a larger request takes the largest)
template <typename T, int p, int NSH, typename F> static inline hipError_t pick(int shv, F&& f) {
  if constexpr (p < 64) {
    return f(IC<0>{});
  } else {
    const int sh = shv & 3, pv = shv >> 2;
    if constexpr (plan_variants<T, p>()) {
      if (pv == 1) return pick_sh<NSH, 1>(sh, f);
      if (pv == 2) return pick_sh<NSH, 2>(sh, f);
    }
    return pick_sh<NSH, 0>(sh, f);
  }
}

template <typename T>
hipError_t launch_fx(int P, bool gen, const T* F, c2<T>* A, const FwdArgs& a, const c2<T>* tw, const Launch& L) {
  switch (P) {
#define X(p)                                                                                                     \
  case p: {                                                                                                      \
    if (gen) return go(k_fx<T, p, true, 0>, dim3(cdiv(a.ny_in, 2 * TileC<T, p, 0>::C), a.nz_in), L, F, A, a, tw); \
    return pick<T, p, 3>(L.sh, [&](auto v) {                                                                     \
      constexpr int S = decltype(v)::value;                                                                      \
      return go(k_fx<T, p, false, S>, dim3(cdiv(a.ny_in, 2 * TileC<T, p, S & 3>::C), a.nz_in), L, F, A, a, tw);  \
    });                                                                                                          \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_fy(int P, bool prune, const c2<T>* A, c2<T>* B, const FwdArgs& a, const c2<T>* tw, const Launch& L) {
  const long long nrows = (long long)a.kx_n * a.nz_in;
  switch (P) {
#define X(p)                                                                                                     \
  case p: {                                                                                                      \
    if (!prune) return go(k_fy<T, p, false, 0>, dim3(cdiv(nrows, TileC<T, p, 0>::C)), L, A, B, a, tw);           \
    return pick<T, p, 3>(L.sh, [&](auto v) {                                                                     \
      constexpr int S = decltype(v)::value;                                                                      \
      return go(k_fy<T, p, true, S>, dim3(cdiv(nrows, TileC<T, p, S & 3>::C)), L, A, B, a, tw);                   \
    });                                                                                                          \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_fz(int P, int mode, const c2<T>* B, c2<T>* S, const FwdArgs& a, const c2<T>* tw, const Launch& L) {
  switch (P) {
#define X(p)                                                                                                     \
  case p: {                                                                                                      \
    if (mode != 0) {                                                                                             \
      dim3 g1(cdiv(a.py / 2 + 1, TileC<T, p, 0>::C), a.kx_n);                                                    \
      return go(k_fz<T, p, 1, 0>, g1, L, B, S, a, tw);                                                           \
    }                                                                                                            \
    int nblk = 0;                                                                                                \
    hipError_t e = pick<T, p, 2>(L.sh, [&](auto v) {                                                             \
      constexpr int SV = decltype(v)::value;                                                                     \
      const long long npr = (cdiv(a.py, TileC<T, p, SV & 3>::C) + 1) / 2;                                        \
      dim3 g(16 * cdiv((long long)a.kx_n * npr, 8));                                                             \
      nblk = (int)g.x;                                                                                           \
      return go(k_fz<T, p, 0, SV>, g, L, B, S, a, tw);                                                           \
    });                                                                                                          \
    if (e != hipSuccess) return e;                                                                               \
    hipLaunchKernelGGL(k_bins_final, dim3(64), dim3(NT), 0, L.s, a, nblk);                                       \
    return hipGetLastError();                                                                                    \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

// grid of the inverse z pass: groups of four tiles (xcd_quad_map)
template <typename T, int p, int SH> static inline dim3 iz_grid(const InvArgs& a) {
  const int C = TileC<T, p, SH >= 1 ? 1 : 0>::C;
  const long long ntile = cdiv(a.py, C);
  const long long ngroups = (long long)a.kx_n * (((ntile + 1) / 2 + 1) / 2);
  return dim3(32 * cdiv(ngroups, 8));
}

template <typename T>
hipError_t launch_iz(int P, int mode, const c2<T>* S, c4<T>* W1, const InvArgs& a, const c2<T>* tw, const Launch& L) {
  switch (P) {
#define X(p)                                                                                                     \
  case p: {                                                                                                      \
    if (mode != 0)                                                                                               \
      return pick<T, p, 2>(L.sh, [&](auto v) {                                                                   \
        constexpr int SV = decltype(v)::value;                                                                   \
        return go(k_iz<T, p, 1, SV, false>, iz_grid<T, p, SV & 3>(a), L, S, W1, a, tw);                          \
      });                                                                                                        \
    const bool k32 = sizeof(T) == 4 && a.oct32 && a.filt != 2; /* TSVD decides its cut in FP64 */            \
    if (a.kmode)                                                                                                 \
      return pick<T, p, 3>(L.sh, [&](auto v) {                                                                   \
        constexpr int SV = decltype(v)::value;                                                                   \
        dim3 g = iz_grid<T, p, SV & 3>(a);                                                                       \
        g.y = cdiv(a.kmax, a.kb);                                                                                \
        if constexpr (sizeof(T) == 4)                                                                            \
          if (k32) return go(k_iz<T, p, 0, SV, true, true>, g, L, S, W1, a, tw);                                 \
        return go(k_iz<T, p, 0, SV, true>, g, L, S, W1, a, tw);                                                  \
      });                                                                                                        \
    return pick<T, p, 3>(L.sh, [&](auto v) {                                                                     \
      constexpr int SV = decltype(v)::value;                                                                     \
      if constexpr (sizeof(T) == 4)                                                                              \
        if (k32) return go(k_iz<T, p, 0, SV, false, true>, iz_grid<T, p, SV & 3>(a), L, S, W1, a, tw);           \
      return go(k_iz<T, p, 0, SV, false>, iz_grid<T, p, SV & 3>(a), L, S, W1, a, tw);                            \
    });                                                                                                          \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T> bool iz_slope_map(int P, int sh, InvArgs& a) {
  switch (P) {
#define X(p)                                                                                                     \
  case p:                                                                                                        \
    (void)pick<T, p, 3>(sh, [&](auto v) {                                                                        \
      constexpr int SV = decltype(v)::value;                                                                     \
      a.slope_n = (int)iz_grid<T, p, SV & 3>(a).x;                                                               \
      a.slope_ntile = (int)cdiv(a.py, TileC<T, p, (SV & 3) >= 1 ? 1 : 0>::C);                                    \
      return hipSuccess;                                                                                         \
    });                                                                                                          \
    return true;
    FR3D_SIZES(X)
#undef X
    default:
      return false;
  }
}

template <typename T>
hipError_t launch_iy(int P, const c4<T>* W1, c4<T>* W2, const InvArgs& a, const c2<T>* tw, const Launch& L) {
  const long long nrows = (long long)a.kx_n * a.nz;
  switch (P) {
#define X(p)                                                                                                     \
  case p: {                                                                                                      \
    return pick<T, p, 3>(L.sh, [&](auto v) {                                                                     \
      constexpr int S = decltype(v)::value;                                                                      \
      dim3 g(cdiv(nrows, TileC<T, p, (S & 3) + 1>::C), a.kmode ? a.kmax : 1);                                    \
      return go(k_iy<T, p, S>, g, L, W1, W2, a, tw);                                                             \
    });                                                                                                          \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t launch_ix(int P, int mode, const c4<T>* W2, T* out, const InvArgs& a, const c2<T>* tw, const Launch& L) {
  switch (P) {
#define X(p)                                                                                                     \
  case p: {                                                                                                      \
    dim3 g;                                                                                                      \
    hipError_t e = pick<T, p, 2>(L.sh, [&](auto v) {                                                             \
      constexpr int S = decltype(v)::value;                                                                      \
      g = dim3(cdiv(a.ny, TileC<T, p, S & 3>::C), a.nz, a.kmode ? a.kmax : 1);                                   \
      return mode != 0 ? go(k_ix<T, p, 1, S>, g, L, W2, out, a, tw) : go(k_ix<T, p, 0, S>, g, L, W2, out, a, tw); \
    });                                                                                                          \
    if (e != hipSuccess || mode != 0) return e;                                                                  \
    if (a.kmode) hipLaunchKernelGGL(k_norm_final_k, dim3(1), dim3(NT), 0, L.s, a, (int)(g.x * g.y));             \
    else hipLaunchKernelGGL(k_norm_final, dim3(1), dim3(NT), 0, L.s, a, (int)(g.x * g.y));                       \
    return hipGetLastError();                                                                                    \
  }
    FR3D_SIZES(X)
#undef X
    default:
      return hipErrorInvalidValue;
  }
}

#define FR3D_INST(T)                                                                                          \
  template hipError_t launch_fx<T>(int, bool, const T*, c2<T>*, const FwdArgs&, const c2<T>*, const Launch&); \
  template hipError_t launch_fy<T>(int, bool, const c2<T>*, c2<T>*, const FwdArgs&, const c2<T>*, const Launch&); \
  template hipError_t launch_fz<T>(int, int, const c2<T>*, c2<T>*, const FwdArgs&, const c2<T>*, const Launch&);  \
  template hipError_t launch_iz<T>(int, int, const c2<T>*, c4<T>*, const InvArgs&, const c2<T>*, const Launch&);  \
  template hipError_t launch_iy<T>(int, const c4<T>*, c4<T>*, const InvArgs&, const c2<T>*, const Launch&);       \
  template bool iz_slope_map<T>(int, int, InvArgs&);                                                              \
  template hipError_t launch_ix<T>(int, int, const c4<T>*, T*, const InvArgs&, const c2<T>*, const Launch&);

}  // namespace fr3d
