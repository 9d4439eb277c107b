// Kernels of the alpha predictor (interface and layouts in mlp.hpp).
//
// Matrix products use V_MFMA_F32_16X16X16_BF16: per 64-lane wavefront, lane l
// supplies A[l%16][4(l/16)+j] and B[4(l/16)+j][l%16] (j = 0..3) and receives
// D[4(l/16)+j][l%16].  Every operand entering a product is rounded to bf16
// (round to nearest even); sums are FP32.
#include "mlp.hpp"

namespace fr3d {
namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }
__device__ __forceinline__ float rbf(float f) { return from_bf16(to_bf16(f)); }

__device__ __forceinline__ float gelu(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float x) {
  return 0.5f * (1.0f + erff(x * 0.70710678118654752f)) + x * 0.39894228040143268f * expf(-0.5f * x * x);
}

__device__ __forceinline__ f32x4 mfma(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// The prediction la (log10 alpha) plus its calibration dc as the first
// point of a seeded search, and the secant slope from the noise feature
// x_64 = log10(delta/||F||).
__device__ __forceinline__ void write_seed(Ctrl* seed, double la, double dc, const float* X) {
  double t = fmin(fmax(la + dc, seed->lo), seed->hi);
  if (t < seed->lo + seed->snap) t = seed->lo;
  seed->t = t;
  seed->alpha_abs = pow(10.0, t) * seed->a_scale;
  seed->state = ST_SEED;
  if (seed->slope > 0 && seed->slope_x != 0)
    seed->slope = fmin(fmax(seed->slope * pow(10.0, seed->slope_x * (double)X[MLP_IN - 1]), 1e-4), 1e3);
}

// ------------------------------------------------------------------ forward
// One row (the seed of a search): the same products (bf16 operands, FP32
// sums) as matrix-vector products over a whole workgroup -- two threads per
// output unit -- instead of one wavefront with 16-row matrix tiles, 15 of
// whose rows would be empty.
__global__ __launch_bounds__(256) void k_mlp_fwd1(const float* __restrict__ p, const float* __restrict__ norm,
                                                  const float* __restrict__ X, float* __restrict__ out, Ctrl* seed,
                                                  const double* __restrict__ cal) {
  __shared__ float xs[MLP_IN], h1[MLP_H], h2[MLP_H], red[4];
  __shared__ double redc[4];
  const int tid = threadIdx.x, j = tid >> 1, hf = tid & 1;
  if (tid < MLP_IN) xs[tid] = rbf((X[tid] - norm[tid]) / norm[MLP_IN + tid]);
  __syncthreads();
  float s = 0.0f;
  for (int k = hf; k < MLP_IN; k += 2) s += rbf(p[OFF_W1 + j * MLP_IN + k]) * xs[k];
  s += __shfl_xor(s, 1, 64);
  if (hf == 0) h1[j] = rbf(gelu(s + p[OFF_B1 + j]));
  __syncthreads();
  s = 0.0f;
  for (int k = hf; k < MLP_H; k += 2) s += rbf(p[OFF_W2 + j * MLP_H + k]) * h1[k];
  s += __shfl_xor(s, 1, 64);
  if (hf == 0) h2[j] = rbf(gelu(s + p[OFF_B2 + j]));
  __syncthreads();
  float v = tid < MLP_H ? h2[tid] * rbf(p[OFF_W3 + tid]) : 0.0f;
  // calibration of the seed: a linear function of the raw features (FP64)
  double vc = (cal && tid < MLP_IN) ? cal[1 + tid] * (double)X[tid] : 0.0;
  for (int off = 32; off > 0; off >>= 1) {
    v += __shfl_xor(v, off, 64);
    vc += __shfl_xor(vc, off, 64);
  }
  if ((tid & 63) == 0) {
    red[tid >> 6] = v;
    redc[tid >> 6] = vc;
  }
  __syncthreads();
  if (tid == 0) {
    const float y = (red[0] + red[1] + red[2] + red[3]) + p[OFF_B3];
    const float la = norm[2 * MLP_IN] + norm[2 * MLP_IN + 1] * y;
    if (out) out[0] = la;
    if (seed) write_seed(seed, (double)la, cal ? cal[0] + ((redc[0] + redc[1]) + (redc[2] + redc[3])) : 0.0, X);
  }
}

// One wavefront per 16 batch rows.
__global__ __launch_bounds__(64) void k_mlp_fwd(const float* __restrict__ p, const float* __restrict__ norm,
                                                const float* __restrict__ X, int B, float* __restrict__ out,
                                                MlpWork w, int train) {
  __shared__ uint16_t xs[16][MLP_INP];
  __shared__ uint16_t hs[16][MLP_H];
  __shared__ float h2s[16][MLP_H];
  const int l = threadIdx.x, li = l & 15, lq = l >> 4;
  const int r0 = blockIdx.x * 16;
  for (int e = l; e < 16 * MLP_INP; e += 64) {
    const int i = e / MLP_INP, k = e % MLP_INP, b = r0 + i;
    float v = 0.0f;
    if (b < B && k < MLP_IN) v = (X[(size_t)b * MLP_IN + k] - norm[k]) / norm[MLP_IN + k];
    const uint16_t hb = to_bf16(v);
    xs[i][k] = hb;
    if (train && b < B) w.xb[(size_t)b * MLP_INP + k] = hb;
  }
  __syncthreads();
  // layer 1: z1 = W1 x + b1
  for (int nt = 0; nt < MLP_H / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int n = nt * 16 + li;
#pragma unroll
    for (int kk = 0; kk < MLP_INP / 16; ++kk) {
      bf16x4 a, bb;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kk * 16 + 4 * lq + j;
        a[j] = (short)xs[li][k];
        bb[j] = (short)(k < MLP_IN ? to_bf16(p[OFF_W1 + n * MLP_IN + k]) : 0);
      }
      acc = mfma(a, bb, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 4 * lq + j, col = nt * 16 + li, b = r0 + row;
      const float z = acc[j] + p[OFF_B1 + col];
      const uint16_t hb = to_bf16(gelu(z));
      hs[row][col] = hb;
      if (train && b < B) {
        w.z1[(size_t)b * MLP_H + col] = z;
        w.h1b[(size_t)b * MLP_H + col] = hb;
      }
    }
  }
  __syncthreads();
  // layer 2: z2 = W2 h1 + b2
  for (int nt = 0; nt < MLP_H / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int n = nt * 16 + li;
#pragma unroll
    for (int kk = 0; kk < MLP_H / 16; ++kk) {
      bf16x4 a, bb;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kk * 16 + 4 * lq + j;
        a[j] = (short)hs[li][k];
        bb[j] = (short)to_bf16(p[OFF_W2 + n * MLP_H + k]);
      }
      acc = mfma(a, bb, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 4 * lq + j, col = nt * 16 + li, b = r0 + row;
      const float z = acc[j] + p[OFF_B2 + col];
      const uint16_t hb = to_bf16(gelu(z));
      h2s[row][col] = from_bf16(hb);
      if (train && b < B) {
        w.z2[(size_t)b * MLP_H + col] = z;
        w.h2b[(size_t)b * MLP_H + col] = hb;
      }
    }
  }
  __syncthreads();
  // layer 3: y = w3 . h2 + b3 (lane li = row, lq = quarter of the 128 inputs)
  float s = 0.0f;
  for (int c = lq * 32; c < lq * 32 + 32; ++c) s += h2s[li][c] * rbf(p[OFF_W3 + c]);
  s += __shfl_xor(s, 16, 64);
  s += __shfl_xor(s, 32, 64);
  if (lq == 0) {
    const int b = r0 + li;
    if (b < B) {
      const float y = s + p[OFF_B3];
      if (train) w.y[b] = y;
      const float la = norm[2 * MLP_IN] + norm[2 * MLP_IN + 1] * y;
      if (out) out[b] = la;

    }
  }
}

// ------------------------------------------------------------------ backward
// Per 16 batch rows: dy = 2 (y - t~)/B, dz2 = q(dy) q(w3) gelu'(z2),
// dh1 = q(dz2) q(W2), dz1 = dh1 gelu'(z1).
__global__ __launch_bounds__(64) void k_mlp_bwd_act(const float* __restrict__ p, const float* __restrict__ norm,
                                                    const float* __restrict__ t, int B, MlpWork w) {
  __shared__ float dys[16];
  __shared__ uint16_t dzs[16][MLP_H];
  const int l = threadIdx.x, li = l & 15, lq = l >> 4;
  const int r0 = blockIdx.x * 16;
  if (l < 16) {
    const int b = r0 + l;
    float d = 0.0f;
    if (b < B) {
      const float tn = (t[b] - norm[2 * MLP_IN]) / norm[2 * MLP_IN + 1];
      const float e = w.y[b] - tn;
      d = 2.0f * e / (float)B;
      w.sq[b] = e * e;
      w.dy[b] = d;
    }
    dys[l] = d;
  }
  __syncthreads();
  for (int e = l; e < 16 * MLP_H; e += 64) {
    const int row = e / MLP_H, c = e % MLP_H, b = r0 + row;
    float dz = 0.0f;
    if (b < B) dz = rbf(dys[row]) * rbf(p[OFF_W3 + c]) * gelu_d(w.z2[(size_t)b * MLP_H + c]);
    const uint16_t hb = to_bf16(dz);
    dzs[row][c] = hb;
    if (b < B) {
      w.dz2[(size_t)b * MLP_H + c] = dz;
      w.dz2b[(size_t)b * MLP_H + c] = hb;
    }
  }
  __syncthreads();
  for (int nt = 0; nt < MLP_H / 16; ++nt) {
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    const int n = nt * 16 + li;
#pragma unroll
    for (int kk = 0; kk < MLP_H / 16; ++kk) {
      bf16x4 a, bb;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int k = kk * 16 + 4 * lq + j;
        a[j] = (short)dzs[li][k];
        bb[j] = (short)to_bf16(p[OFF_W2 + k * MLP_H + n]);
      }
      acc = mfma(a, bb, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int row = 4 * lq + j, col = nt * 16 + li, b = r0 + row;
      if (b < B) {
        const float dz = acc[j] * gelu_d(w.z1[(size_t)b * MLP_H + col]);
        w.dz1[(size_t)b * MLP_H + col] = dz;
        w.dz1b[(size_t)b * MLP_H + col] = to_bf16(dz);
      }
    }
  }
}

// Weight gradients, one wavefront per 16x16 tile with the batch as the
// reduction axis: blocks [0,64) dW2 = q(dz2)^T q(h1), [64,104) dW1 =
// q(dz1)^T q(x); block 104: db1, db2, dw3 = q(h2)^T q(dy), db3 and the loss.
__global__ __launch_bounds__(64) void k_mlp_wgrad(int B, MlpWork w, float* __restrict__ grad, float* loss) {
  const int l = threadIdx.x, li = l & 15, lq = l >> 4;
  const int id = blockIdx.x;
  if (id < 104) {
    const bool l2 = id < 64;
    const int mt = l2 ? id / 8 : (id - 64) / 5, nt = l2 ? id % 8 : (id - 64) % 5;
    const uint16_t* A = l2 ? w.dz2b : w.dz1b;
    const uint16_t* Bm = l2 ? w.h1b : w.xb;
    const int ldb = l2 ? MLP_H : MLP_INP;
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    for (int b0 = 0; b0 < B; b0 += 16) {
      bf16x4 a, bb;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int b = b0 + 4 * lq + j;
        a[j] = (short)(b < B ? A[(size_t)b * MLP_H + mt * 16 + li] : 0);
        bb[j] = (short)(b < B ? Bm[(size_t)b * ldb + nt * 16 + li] : 0);
      }
      acc = mfma(a, bb, acc);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int n = mt * 16 + 4 * lq + j, k = nt * 16 + li;
      if (l2) grad[OFF_W2 + n * MLP_H + k] = acc[j];
      else if (k < MLP_IN) grad[OFF_W1 + n * MLP_IN + k] = acc[j];
    }
    return;
  }
  for (int c = l; c < MLP_H; c += 64) {
    float s1 = 0.f, s2 = 0.f, s3 = 0.f;
    for (int b = 0; b < B; ++b) {
      s1 += w.dz1[(size_t)b * MLP_H + c];
      s2 += w.dz2[(size_t)b * MLP_H + c];
      s3 += from_bf16(w.h2b[(size_t)b * MLP_H + c]) * rbf(w.dy[b]);
    }
    grad[OFF_B1 + c] = s1;
    grad[OFF_B2 + c] = s2;
    grad[OFF_W3 + c] = s3;
  }
  if (l == 0) {
    float s = 0.f, q = 0.f;
    for (int b = 0; b < B; ++b) {
      s += w.dy[b];
      q += w.sq[b];
    }
    grad[OFF_B3] = s;
    if (loss) *loss = q / (float)B;
  }
}

__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                       float* __restrict__ v, float lr, float c1, float c2) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= MLP_NP) return;
  const float gi = g[i];
  const float mi = 0.9f * m[i] + 0.1f * gi;
  const float vi = 0.999f * v[i] + 0.001f * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + 1e-8f);
}

}  // namespace

size_t mlp_work_bytes(int cap) {
  const size_t c = (size_t)cap;
  return c * MLP_INP * 2 + c * MLP_H * (4 + 2 + 4 + 2 + 4 + 2 + 4 + 2) + c * 4 * 3 + 1024;
}

void mlp_work_carve(MlpWork* w, void* base, int cap) {
  char* q = (char*)base;
  const size_t c = (size_t)cap;
  auto take = [&](size_t bytes) {
    char* r = q;
    q += (bytes + 255) & ~(size_t)255;
    return (void*)r;
  };
  w->cap = cap;
  w->xb = (uint16_t*)take(c * MLP_INP * 2);
  w->z1 = (float*)take(c * MLP_H * 4);
  w->h1b = (uint16_t*)take(c * MLP_H * 2);
  w->z2 = (float*)take(c * MLP_H * 4);
  w->h2b = (uint16_t*)take(c * MLP_H * 2);
  w->dz1 = (float*)take(c * MLP_H * 4);
  w->dz1b = (uint16_t*)take(c * MLP_H * 2);
  w->dz2 = (float*)take(c * MLP_H * 4);
  w->dz2b = (uint16_t*)take(c * MLP_H * 2);
  w->y = (float*)take(c * 4);
  w->dy = (float*)take(c * 4);
  w->sq = (float*)take(c * 4);
}

hipError_t mlp_forward(const float* params, const float* norm, const float* X, int B, float* out, MlpWork* w,
                       Ctrl* seed, hipStream_t s, const double* cal) {
  if (B <= 0 || (w && B > w->cap) || (seed && (B != 1 || w))) return hipErrorInvalidValue;
  if (seed) {
    hipLaunchKernelGGL(k_mlp_fwd1, dim3(1), dim3(256), 0, s, params, norm, X, out, seed, cal);
    return hipGetLastError();
  }
  MlpWork dummy{};
  hipLaunchKernelGGL(k_mlp_fwd, dim3((B + 15) / 16), dim3(64), 0, s, params, norm, X, B, out, w ? *w : dummy,
                     w ? 1 : 0);
  return hipGetLastError();
}

hipError_t mlp_backward_adam(float* params, const float* norm, const float* t, int B, MlpWork* w, float* grad,
                             float* loss, float* m, float* v, double lr, double c1, double c2, hipStream_t s) {
  if (B <= 0 || !w || B > w->cap) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_mlp_bwd_act, dim3((B + 15) / 16), dim3(64), 0, s, params, norm, t, B, *w);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mlp_wgrad, dim3(105), dim3(64), 0, s, B, *w, grad, loss);
  e = hipGetLastError();
  if (e != hipSuccess || !(lr > 0)) return e;
  hipLaunchKernelGGL(k_adam, dim3((MLP_NP + 255) / 256), dim3(256), 0, s, params, grad, m, v, (float)lr, (float)c1,
                     (float)c2);
  return hipGetLastError();
}

}  // namespace fr3d
