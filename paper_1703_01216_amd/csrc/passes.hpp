// Pencil passes of the zero-padded 3D transforms and their fused prologues and
// epilogues (Algorithm 1, steps 1-3, Sec. 4, with the transform over all three
// axes of the P^3 = (2n)^3 box).
//
// Volume layouts in device memory (T = float or double, c2 = complex T):
//   F, zeta      real  [nz][ny][nx]                 data on Y / estimate on R
//   A  (x done)  c2    [Kx][nz][ny]     Kx = Px/2+1 real-to-complex along x
//   B  (y done)  c2    [Kx][nz][Py]
//   S  (spectrum)c2    [Kx][Py/G][Pz][G] f^ for kx <= Px/2 (f is real), in
//                                       column granules (spec_lg below)
//   O  (octant)  double2 [Kx][Pz/2+1][Py/2+1]   k^ (even in kx, ky; Hermitian in kz)
//   W1 (z undone) c4   [Kx][nz][Py]     (u^, r^) pairs, z < nz only
//   W2 (y undone) c4   [Kx][nz][ny]
// The forward passes read only the n nonzero inputs of each pencil; the
// inverse passes write only the outputs inside R / Y.  The x axis is the
// slowest axis of every spectral volume, so the y pass reads and writes whole
// rows and the z and x passes read rows of C consecutive pencils.
#pragma once

#include "control.hpp"
#include "fft_core.hpp"

namespace fr3d {

constexpr int NT = 256;  // threads per workgroup of every pass

// Pencils per workgroup: a 32 KiB tile (FP32: 4096 elements, FP64: 2048),
// halved SH times (the tile-size variants the autotuner chooses from).
template <typename T, int P> struct Tile {
  static constexpr int pow2ceil(int v) { int p = 1; while (p < v) p <<= 1; return p; }
  static constexpr int TE = sizeof(T) == 4 ? 4096 : 2048;
  static constexpr int C = TE / pow2ceil(P) > 0 ? TE / pow2ceil(P) : 1;
};
template <typename T, int P, int SH> struct TileC {
  static constexpr int C = (Tile<T, P>::C >> SH) > 0 ? (Tile<T, P>::C >> SH) : 1;
};

// Column granules of the spectrum S: the Py columns of a kx plane are cut
// into granules of G = 2^lg consecutive ky, and a granule's rows kz = 0..Pz-1
// are stored one after another, so f^(kx, kz, ky) sits at
//   ((kx ng + ky / G) Pz + kz) G + ky mod G,   ng = ceil(Py / G).
// G is the column count of the z passes' half tile (which divides every
// z-pass tile width), at most the largest power of two <= Py: every z-pass
// workgroup then reads or writes whole granules, i.e. contiguous blocks,
// instead of short column segments at the row pitch.  Columns ky >= Py of a
// last, partial granule are never written or read.
__host__ __device__ inline int spec_lg(int esz, int pz, int py) {
  int p2 = 1;
  while (p2 < pz) p2 <<= 1;
  int c1 = (esz == 4 ? 4096 : 2048) / p2;  // Tile<T, Pz>::C
  c1 = c1 > 0 ? c1 : 1;
  c1 = (c1 >> 1) > 0 ? (c1 >> 1) : 1;  // TileC<T, Pz, 1>::C
  int lg = 0;
  while ((2 << lg) <= py && (2 << lg) <= c1) ++lg;
  return lg;
}
__host__ __device__ inline int spec_ng(int py, int lg) { return (py + (1 << lg) - 1) >> lg; }
// Offset of (kz, ky) within a kx plane of S.
__host__ __device__ inline size_t spec_off(int kz, int ky, int pz, int lg) {
  return ((((size_t)(ky >> lg) * pz) + kz) << lg) + (ky & ((1 << lg) - 1));
}
// Elements of one kx plane of S (padding columns included).
__host__ __device__ inline size_t spec_plane(int pz, int py, int lg) { return ((size_t)spec_ng(py, lg) * pz) << lg; }

// Padded box of the predictor features' energies (Parseval normalisation,
// half-spectrum weights).
struct BinGeom {
  int px, py, pz;
};

struct FwdArgs {
  int nz_in, ny_in;   // rows of the x pass: nz_in planes of ny_in rows
  int kx_n;           // Px/2 + 1
  int py, pz;         // padded extents
  // kernel sampling (x pass in generator mode)
  double h, hz, D;    // lateral and vertical cell edges, gap in vertical cells
  int nx, ny, nz;     // cell counts
  int kind;
  int zlin;           // generator mode: plane z samples the z offset z - (nz - 1) (no wrap)
  const double* ksrc; // generator mode: read the wrapped samples [Pz][Py][Px] from here instead
  // energy epilogue
  BinGeom bg;
  // level of the kernel spectrum per (kx, |ky|, kz), [kx][Py/2+1][Pz] (kz
  // fastest): the number of thresholds s_max 10^((j - 64)/4), j = 1..63,
  // that |k^|^2 reaches; a data point's energy goes to its level's bin
  const uint8_t* level;
  double* bins_part;  // [64][z-pass workgroups]
  double* bins_out;   // [64] energies
  float* feat_out;    // [65] features
  uint32_t* ticket;
  double delta;       // noise level for the last feature
};

struct InvArgs {
  int nx, ny, nz;
  int kx_n, py, pz;
  double scale;             // 1/(Px Py Pz)
  const double2* oct;
  const float2* oct32;      // the octant rounded to FP32 (FP32 contexts; the FP32 Tikhonov-family filter)
  Ctrl* ctrl;               // null for the forward operator (no search)
  double2* norm_part;       // [x-pass workgroups] (||r||^2, ||zeta||^2) partials
  // K-candidate step (kmode = 1): candidate j filters with ctrl->ca[j] and
  // works in its own slices W1 + j w1_stride, W2 + j w2_stride and
  // norm_part + j norm_stride; zeta is not written.  The passes of a
  // K-candidate step run only while the search is in that state, the passes
  // of a single evaluation only while it is not.
  int adj;                  // forward-operator mode: 1 applies the adjoint (conjugate spectrum)
  int filt;                 // regularising filter: 0 Tikhonov, 1 iterated Tikhonov, 2 truncated SVD
  int order;                // order of iterated Tikhonov (>= 1)
  int kmode;
  int kmax;                 // K (grid extent over candidates)
  int kb;                   // candidates per z-pass workgroup
  long long w1_stride, w2_stride, norm_stride;
  // single evaluations with diagnostics: per-workgroup partial sums of the
  // full-box residual (Parseval over the half spectrum); null: not formed
  double* full_part;
  // the seed evaluation of a secant search with a slope ratio (Tikhonov
  // filter): per wave of each z-pass workgroup, [workgroup][NT / 64],
  // (sum w e^2 |f^|^2, sum w e^2 (1 - e) |f^|^2) over its points,
  // e = a / (s + a) the residual factor and w the half-spectrum weight; the
  // x pass's final kernel forms the full-box slope from the entries of the
  // workgroups that hold a tile.  Set for the seed's launch only; null
  // otherwise.
  double2* slope_part;
  int slope_n;              // z-pass workgroups
  int slope_ntile;          // column tiles per kx plane of the z pass
};

// Whether an inverse-pass kernel of this launch has nothing to do; alpha:
// the single evaluation's filter alpha (one load with the state).
__device__ __forceinline__ bool inv_idle(const InvArgs& a, double& alpha) {
  alpha = 0.0;
  if (!a.ctrl) return false;
  int32_t state, active;
  ctrl_head(a.ctrl, state, active, alpha);
  return !active || ((state == ST_KARY) != (a.kmode != 0));
}
__device__ __forceinline__ bool inv_idle(const InvArgs& a) {
  double alpha;
  return inv_idle(a, alpha);
}

// ------------------------------------------------------------------ host launchers
// Stream and, when timing, the event pair recorded at the pass kernel's start
// and end (hipExtLaunchKernel).
struct Launch {
  hipStream_t s;
  hipEvent_t e0, e1;
  int sh;  // tile-size variant (0 = 32 KiB tile, 1 = half, 2 = quarter (row passes)) + 4 x the radix
           // plan variant (0-2; FP32 lengths 192, 384 and 512)
};

// Each returns hipSuccess or the launch error; P is the transform length of
// the pass axis and selects the compiled instance.
template <typename T>
hipError_t launch_fx(int P, bool gen, const T* F, c2<T>* A, const FwdArgs& a, const c2<T>* tw, const Launch& L);
template <typename T>
hipError_t launch_fy(int P, bool prune, const c2<T>* A, c2<T>* B, const FwdArgs& a, const c2<T>* tw, const Launch& L);
// mode 0: data (pruned input, full output, energy partials + final features kernel);
// mode 1: kernel (full input, octant output)
template <typename T>
hipError_t launch_fz(int P, int mode, const c2<T>* B, c2<T>* S, const FwdArgs& a, const c2<T>* tw, const Launch& L);
// mode 0: Tikhonov filter (u^, r^); 1: multiply by k^ (forward operator).
// With a.kmode the z, y and x passes cover a.kmax candidates (a grid
// dimension) and the x pass is followed by the K-way norm kernel.
template <typename T>
hipError_t launch_iz(int P, int mode, const c2<T>* S, c4<T>* W1, const InvArgs& a, const c2<T>* tw, const Launch& L);
template <typename T>
hipError_t launch_iy(int P, const c4<T>* W1, c4<T>* W2, const InvArgs& a, const c2<T>* tw, const Launch& L);
// The workgroup map of launch_iz's single-evaluation Tikhonov launch for
// tile code sh, into a.slope_n and a.slope_ntile; false for an
// unsupported length.
template <typename T>
bool iz_slope_map(int P, int sh, InvArgs& a);
template <typename T>
hipError_t launch_ix(int P, int mode, const c4<T>* W2, T* out, const InvArgs& a, const c2<T>* tw, const Launch& L);

bool supported_length(int P);

}  // namespace fr3d
