// Algorithm 1 with the per-frequency z-systems of Sec. 5, Eq. (14): after the
// lateral 2D transform, every lateral frequency (kx, ky) has a real M x M
// system A[i][j] = k~(kx, ky; i - j) between the M layers of R and of Y,
// where k~(.; dz) is the lateral transform of the kernel samples at the z
// offset (D + dz) h.  K is even in x and y, so A depends on (kx, |ky|) only
// and is real.  The systems are regularised through their SVD A = U S V^T
// (computed once per geometry by one-sided Jacobi rotations); an evaluation
// at alpha forms, per frequency,
//   w = A^T f^,  b = V^T w,  x^ = V diag(h(s^2, alpha)) b,  r^ = A x^ - f^
// with h = phi(s)/s^2 from the filter factors phi of Tikhonov, iterated
// Tikhonov or TSVD, and writes (x^, r^) in the inverse passes' W1 layout,
// so the lateral inverse passes, the norms and the alpha search are shared
// with the 3D path.
//
// Layouts (f = kx * (Py/2 + 1) + |ky| indexes the distinct systems):
//   kt   double [f][2M - 1]   A's Toeplitz entries, kt[f][i - j + M - 1]
//   V    double [f][M][M]     right singular vectors, V[i][k]
//   lam  double [f][M]        squared singular values s_k^2
//   B    c2<T>  [Kx][M][Py]   lateral spectrum of each layer (data or zeta)
#pragma once

#include "passes.hpp"

namespace fr3d {

constexpr int LAY_MMAX = 60;  // layers per system (both matrices of the SVD fit one workgroup's LDS)

struct LayArgs {
  int M;            // layers of R and of Y
  int kxn, py, pyh; // Px/2 + 1, Py, Py/2 + 1
  const double* kt;
  const double* V;
  const double* lam;
};

// SVD of every distinct system from the lateral kernel transform Bk
// ([Kx][2M-1][Py] complex double); fills kt, V and lam.
hipError_t launch_lay_svd(const double2* Bk, const LayArgs& la, double* kt, double* V, double* lam, hipStream_t s);

// Per-frequency step of an evaluation (mode 0, filter of a.filt with the
// search's alpha, or the K candidates of a K-candidate step) or of the
// forward operator (mode 1: W1 = (A x^, 0) for x^ the lateral spectrum of
// zeta in B).
template <typename T>
hipError_t launch_lay_filter(int mode, const c2<T>* B, c4<T>* W1, const LayArgs& la, const InvArgs& a,
                             const Launch& L);

// Per-frequency alphas (Algorithm 1 step 2 read per lateral frequency): for
// each frequency, the plain discrepancy rule (upper end, lower end, then
// bisection in log10 alpha, any point within tol accepted) on that system's
// residual ||A x^ - f^||, evaluated in closed form from the SVD,
//   ||A x - f||^2 = ||f||^2 - sum_k (2 h_k - s_k^2 h_k^2) |b_k|^2,
// against target = tau delta (unnormalised lateral DFT units); then that
// frequency's (x^, r^) as in k_lay_filter.  Per system partials
// part[5 f + (0..4)] = (sum log10 alpha, frequencies, NOROOT_HIGH count,
// NOROOT_LOW count, MAXITER count), counted over the full Px x Py spectrum;
// alpha_out / flags_out [Kx][Py] optional.
struct PfArgs {
  double target, a_scale, lo, hi, tol;
  int max_steps;
  double* alpha_out;
  int* flags_out;
  double* part;
};
template <typename T>
hipError_t launch_lay_pf(const c2<T>* B, c4<T>* W1, const LayArgs& la, const InvArgs& a, const PfArgs& pf,
                         const Launch& L);

// Singular values s_k = sqrt(lam_k) of every distinct system, descending:
// out[f][k], f = kx (Py/2 + 1) + |ky|.
hipError_t launch_lay_sv(const LayArgs& la, double* out, hipStream_t s);

// max lam (the squared operator norm) into *out (device), via partials.
hipError_t launch_lay_max(const double* lam, long long n, double* part, double* out, hipStream_t s);

}  // namespace fr3d
