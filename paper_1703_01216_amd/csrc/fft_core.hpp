// Device building blocks of the pencil FFTs: complex arithmetic, small DFT
// codelets (radix 2, 3, 4, 8, 16), the radix plan of each transform length and
// an in-LDS Stockham transform over a tile of pencils.
//
// Transform convention: forward X[k] = sum_j x[j] e^{-2 pi i jk/P} (DIR = -1),
// inverse unnormalised with e^{+2 pi i jk/P} (DIR = +1); callers apply 1/P^3.
//
// Stockham autosort (decimation in time): stage s of radix R with Ns the
// product of the earlier radices treats butterfly j in [0, P/R):
//   k = j mod Ns;  v_r = x[j + r P/R] * W_{Ns R}^{r k}  (r < R);  v = DFT_R(v);
//   y[(j div Ns) Ns R + k + r Ns] = v_r.
// The output of the last stage is in natural order.  Each stage reads the
// tile from LDS into registers, synchronises, and writes it back in place.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fr3d {

template <typename T> struct V2;
template <> struct V2<float> { using type = float2; };
template <> struct V2<double> { using type = double2; };
template <typename T> using c2 = typename V2<T>::type;

template <typename T> struct V4;
template <> struct V4<float> { using type = float4; };
template <> struct V4<double> { using type = double4; };
template <typename T> using c4 = typename V4<T>::type;

template <typename T> __device__ __forceinline__ c2<T> mk(T x, T y) { c2<T> r; r.x = x; r.y = y; return r; }
template <typename T> __device__ __forceinline__ c2<T> add(c2<T> a, c2<T> b) { return mk<T>(a.x + b.x, a.y + b.y); }
template <typename T> __device__ __forceinline__ c2<T> sub(c2<T> a, c2<T> b) { return mk<T>(a.x - b.x, a.y - b.y); }
template <typename T> __device__ __forceinline__ c2<T> mul(c2<T> a, c2<T> b) {
  return mk<T>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T> __device__ __forceinline__ c2<T> scl(c2<T> a, T s) { return mk<T>(a.x * s, a.y * s); }
template <typename T> __device__ __forceinline__ c2<T> cj(c2<T> a) { return mk<T>(a.x, -a.y); }
// multiply by DIR * i
template <int DIR, typename T> __device__ __forceinline__ c2<T> rot(c2<T> a) {
  return DIR > 0 ? mk<T>(-a.y, a.x) : mk<T>(a.y, -a.x);
}

// ---------------------------------------------------------------- codelets
template <int DIR, typename T> __device__ __forceinline__ void dft2(c2<T>* v) {
  c2<T> a = v[0], b = v[1];
  v[0] = add<T>(a, b);
  v[1] = sub<T>(a, b);
}

template <int DIR, typename T> __device__ __forceinline__ void dft3(c2<T>* v) {
  const T h = (T)0.86602540378443864676;  // sqrt(3)/2
  c2<T> a = v[0], s = add<T>(v[1], v[2]), d = sub<T>(v[1], v[2]);
  c2<T> m = mk<T>(a.x - (T)0.5 * s.x, a.y - (T)0.5 * s.y);
  c2<T> t = rot<DIR, T>(scl<T>(d, h));
  v[0] = add<T>(a, s);
  v[1] = add<T>(m, t);
  v[2] = sub<T>(m, t);
}

template <int DIR, typename T> __device__ __forceinline__ void dft4(c2<T>& a, c2<T>& b, c2<T>& c, c2<T>& d) {
  c2<T> s0 = add<T>(a, c), d0 = sub<T>(a, c), s1 = add<T>(b, d), d1 = rot<DIR, T>(sub<T>(b, d));
  a = add<T>(s0, s1);
  c = sub<T>(s0, s1);
  b = add<T>(d0, d1);
  d = sub<T>(d0, d1);
}
template <int DIR, typename T> __device__ __forceinline__ void dft4(c2<T>* v) { dft4<DIR, T>(v[0], v[1], v[2], v[3]); }

template <int DIR, typename T> __device__ __forceinline__ void dft8(c2<T>* v) {
  const T r = (T)0.70710678118654752440;
  c2<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  c2<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR, T>(e0, e1, e2, e3);
  dft4<DIR, T>(o0, o1, o2, o3);
  // W8^1 = r(1 + DIR i), W8^2 = DIR i, W8^3 = r(-1 + DIR i)
  o1 = scl<T>(add<T>(o1, rot<DIR, T>(o1)), r);
  o2 = rot<DIR, T>(o2);
  o3 = scl<T>(sub<T>(rot<DIR, T>(o3), o3), r);
  v[0] = add<T>(e0, o0); v[4] = sub<T>(e0, o0);
  v[1] = add<T>(e1, o1); v[5] = sub<T>(e1, o1);
  v[2] = add<T>(e2, o2); v[6] = sub<T>(e2, o2);
  v[3] = add<T>(e3, o3); v[7] = sub<T>(e3, o3);
}

template <int DIR, typename T> __device__ __forceinline__ void dft16(c2<T>* v) {
  const T c1 = (T)0.92387953251128675613, s1 = (T)0.38268343236508977173, r = (T)0.70710678118654752440;
  c2<T> e[8], o[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) { e[i] = v[2 * i]; o[i] = v[2 * i + 1]; }
  dft8<DIR, T>(e);
  dft8<DIR, T>(o);
  const T d = (T)DIR;
  // W16^k = cos(2 pi k/16) + DIR i sin(2 pi k/16)
  const c2<T> w[8] = {mk<T>(1, 0),  mk<T>(c1, d * s1),  mk<T>(r, d * r),  mk<T>(s1, d * c1),
                      mk<T>(0, d),  mk<T>(-s1, d * c1), mk<T>(-r, d * r), mk<T>(-c1, d * s1)};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    c2<T> t = k == 0 ? o[0] : (k == 4 ? rot<DIR, T>(o[4]) : mul<T>(o[k], w[k]));
    v[k] = add<T>(e[k], t);
    v[k + 8] = sub<T>(e[k], t);
  }
}

template <int R, int DIR, typename T> __device__ __forceinline__ void dftR(c2<T>* v) {
  if constexpr (R == 2) dft2<DIR, T>(v);
  else if constexpr (R == 3) dft3<DIR, T>(v);
  else if constexpr (R == 4) dft4<DIR, T>(v);
  else if constexpr (R == 8) dft8<DIR, T>(v);
  else if constexpr (R == 16) dft16<DIR, T>(v);
}

// ---------------------------------------------------------------- radix plans
// Stage radices of each supported length, largest first (variant 0), and
// alternative orders of the three-stage lengths 192, 384 and 512 (variants 1
// and 2), among which the autotuner chooses per pass.
template <int P, int V = 0> struct Plan {  // a length without that variant: the default plan
  static constexpr int nst = Plan<P, 0>::nst, r0 = Plan<P, 0>::r0, r1 = Plan<P, 0>::r1, r2 = Plan<P, 0>::r2;
};
#define FR3D_PLAN(P_, V_, N_, R0, R1, R2)                      \
  template <> struct Plan<P_, V_> {                             \
    static constexpr int nst = N_;                              \
    static constexpr int r0 = R0, r1 = R1, r2 = R2;             \
  };
FR3D_PLAN(4, 0, 1, 4, 1, 1)
FR3D_PLAN(6, 0, 2, 3, 2, 1)
FR3D_PLAN(8, 0, 1, 8, 1, 1)
FR3D_PLAN(12, 0, 2, 4, 3, 1)
FR3D_PLAN(16, 0, 1, 16, 1, 1)
FR3D_PLAN(24, 0, 2, 8, 3, 1)
FR3D_PLAN(32, 0, 2, 8, 4, 1)
FR3D_PLAN(48, 0, 2, 16, 3, 1)
FR3D_PLAN(64, 0, 2, 8, 8, 1)
FR3D_PLAN(96, 0, 3, 8, 4, 3)
FR3D_PLAN(128, 0, 2, 16, 8, 1)
FR3D_PLAN(192, 0, 3, 16, 4, 3)
FR3D_PLAN(192, 1, 3, 8, 8, 3)
FR3D_PLAN(192, 2, 3, 4, 16, 3)
FR3D_PLAN(256, 0, 2, 16, 16, 1)
FR3D_PLAN(384, 0, 3, 16, 8, 3)
FR3D_PLAN(384, 1, 3, 8, 16, 3)
FR3D_PLAN(384, 2, 3, 3, 16, 8)
FR3D_PLAN(512, 0, 3, 8, 8, 8)
FR3D_PLAN(512, 1, 3, 16, 8, 4)
FR3D_PLAN(512, 2, 3, 16, 16, 2)
#undef FR3D_PLAN

// ---------------------------------------------------------------- LDS tile transform
// A tile holds NC pencils of length P in LDS.  COLFAST: element (col, p) at
// p*LD + col (pencils interleaved, column index fastest); otherwise at
// col*LD + rsw(p) (pencils contiguous, bank-skewed).  NT threads cooperate.
// Row layout: element p of a pencil sits at p + p/16, so the stride-R
// stores of a Stockham stage (R <= 16) fall on distinct LDS banks; the row
// pitch LD must then be >= RowLD<P>.
__device__ __forceinline__ int rsw(int p) { return p + (p >> 4); }
template <int P> struct RowLD { static constexpr int value = P + P / 16 + 1; };

template <bool COLFAST, int LD> __device__ __forceinline__ int tile_addr(int col, int p) {
  return COLFAST ? p * LD + col : col * LD + rsw(p);
}

template <typename T, int P, int NC, int LD, int NT, bool COLFAST, int DIR, int R, int NS>
__device__ __forceinline__ void stockham_stage(c2<T>* lds, const c2<T>* tw, int tid) {
  constexpr int NBF = NC * (P / R);  // butterflies in the tile
  constexpr int NB = (NBF + NT - 1) / NT;
  constexpr int M = P / R;
  c2<T> v[NB][R];
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int t = tid + b * NT;
    if (NBF % NT == 0 || t < NBF) {
      const int col = COLFAST ? t % NC : t / M;
      const int j = COLFAST ? t / NC : t % M;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = lds[tile_addr<COLFAST, LD>(col, j + r * M)];
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < NB; ++b) {
    const int t = tid + b * NT;
    if (NBF % NT == 0 || t < NBF) {
      const int col = COLFAST ? t % NC : t / M;
      const int j = COLFAST ? t / NC : t % M;
      const int k = j % NS;
      if constexpr (NS > 1) {
        constexpr int STR = P / (NS * R);
#pragma unroll
        for (int r = 1; r < R; ++r) {
          c2<T> w = tw[(r * k * STR) % P];
          if (DIR > 0) w.y = -w.y;
          v[b][r] = mul<T>(v[b][r], w);
        }
      }
      dftR<R, DIR, T>(v[b]);
      const int base = (j / NS) * NS * R + k;
#pragma unroll
      for (int r = 0; r < R; ++r) lds[tile_addr<COLFAST, LD>(col, base + r * NS)] = v[b][r];
    }
  }
  __syncthreads();
}

// Full transform of the tile; the tile must be in LDS and synchronised on entry.
// tw: the P-entry table e^{-2 pi i m/P} (LDS or global).
template <typename T, int P, int NC, int LD, int NT, bool COLFAST, int DIR, int V = 0>
__device__ __forceinline__ void tile_fft(c2<T>* lds, const c2<T>* tw, int tid) {
  using PL = Plan<P, V>;
  stockham_stage<T, P, NC, LD, NT, COLFAST, DIR, PL::r0, 1>(lds, tw, tid);
  if constexpr (PL::nst > 1) stockham_stage<T, P, NC, LD, NT, COLFAST, DIR, PL::r1, PL::r0>(lds, tw, tid);
  if constexpr (PL::nst > 2)
    stockham_stage<T, P, NC, LD, NT, COLFAST, DIR, PL::r2, PL::r0 * PL::r1>(lds, tw, tid);
}

// Twiddle table into LDS: tw[m] = e^{-2 pi i m / P}, read from the global
// FP64-generated table of this length.
template <typename T, int P, int NT>
__device__ __forceinline__ void load_twiddles(c2<T>* tw_lds, const c2<T>* tw_glob, int tid) {
  for (int m = tid; m < P; m += NT) tw_lds[m] = tw_glob[m];
}

// ---------------------------------------------------------------- reductions
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Sum of p[k es] over k = i0, i0 + st, i0 + 2 st, ... below n, in that order,
// with the loads of U terms issued before any of them is added: the same
// sum as the plain loop, one memory round trip per U terms instead of per
// term (the fixed-order reductions of per-workgroup partials).
__device__ __forceinline__ void acc(double& s, double v) { s += v; }
__device__ __forceinline__ void acc(double2& s, double2 v) { s.x += v.x; s.y += v.y; }
template <typename V, int U = 8>
__device__ __forceinline__ V strided_sum(const V* __restrict__ p, int i0, int n, int st, long long es = 1) {
  V s{};
  for (int b = i0; b < n; b += U * st) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int k = b + u * st;
      if (k < n) v[u] = p[(long long)k * es];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (b + u * st < n) acc(s, v[u]);
  }
  return s;
}

// Sum over the block (NT threads, NT/64 waves), result valid in thread 0.
template <int NT> __device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum<double>(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) red[w] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int i = 0; i < NT / 64; ++i) s += red[i];
  }
  return s;
}

}  // namespace fr3d
