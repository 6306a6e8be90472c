// MLP surrogate for the smooth part L_d(x; k, alpha1, alpha2) of the 3D
// Green's function in the near region (|x3| <= c): L_d = K_d - F, the function
// whose grid values Algorithm 3.1 interpolates.  Network: 64 features -> 4
// hidden layers of 256 (GELU) -> 2 outputs (Re, Im of 10 L_d).  BF16 operands,
// FP32 accumulation on the matrix cores (v_mfma_f32_16x16x16_bf16); FP32
// master weights and Adam moments.
//
// A G_d value from the network is e^{i alpha.x'} L_NN(t) + e^{i 2 pi alpha.n} psi(t)
// with the singular part psi = e^{ikr} Y_eps(r) / (4 pi r) added in FP64, as in
// Algorithm 3.1 step 2e.
#include <cstddef>

#include "qpgf_internal.h"

namespace qpgf {

namespace {

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
constexpr double kPi = 3.141592653589793238462643383279502884;

// ---------------------------------------------------------------------------
// C[M x N] (+)= A[M x K] B[K x N] with arbitrary strides, bf16 in, fp32 out.
// Block tile 64 x 64, four waves of 32 x 32 (2 x 2 MFMA 16x16x16 tiles),
// K in steps of 16 staged through LDS.  blockIdx.z splits K: split z writes
// C + z * c_split (partial sums reduced later).
// ---------------------------------------------------------------------------
struct GemmArgs {
  const __bf16* A;
  long a_m, a_k;
  const __bf16* B;
  long b_k, b_n;
  float* C;
  long c_m, c_n, c_split;
  const float* bias;   // added to column n (split 0 only), may be null
  int M, N, K, ksplit;
};

__global__ __launch_bounds__(256) void k_gemm_bf16(GemmArgs g) {
  __shared__ __bf16 As[64][16 + 4];
  __shared__ __bf16 Bs[16][64 + 4];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  const int kz0 = blockIdx.z * g.ksplit, kz1 = min(g.K, kz0 + g.ksplit);
  const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int k0 = kz0; k0 < kz1; k0 += 16) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = tid * 4 + e;
      const int am = idx >> 4, ak = idx & 15;
      As[am][ak] = g.A[(long)(m0 + am) * g.a_m + (long)(k0 + ak) * g.a_k];
      const int bk = idx >> 6, bn = idx & 63;
      Bs[bk][bn] = g.B[(long)(k0 + bk) * g.b_k + (long)(n0 + bn) * g.b_n];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      bf16x4 a;
#pragma unroll
      for (int r = 0; r < 4; ++r) a[r] = As[wm + 16 * i + (lane & 15)][4 * (lane >> 4) + r];
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        bf16x4 b;
#pragma unroll
        for (int r = 0; r < 4; ++r) b[r] = Bs[4 * (lane >> 4) + r][wn + 16 * j + (lane & 15)];
        acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc[i][j], 0, 0, 0);
      }
    }
    __syncthreads();
  }
  float* C = g.C + (long)blockIdx.z * g.c_split;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + 16 * j + (lane & 15);
      const float bb = (g.bias && blockIdx.z == 0) ? g.bias[n] : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
        C[(long)m * g.c_m + (long)n * g.c_n] = acc[i][j][r] + bb;
      }
    }
}

__device__ __forceinline__ float gelu(float z) { return 0.5f * z * (1.f + erff(z * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_d(float z) {
  return 0.5f * (1.f + erff(z * 0.70710678118654752f)) + z * 0.39894228040143268f * expf(-0.5f * z * z);
}

// A = gelu(Z) in bf16 (row-major) and its transpose AT [N x M]
__global__ void k_gelu_fwd(const float* __restrict__ Z, long M, int N, __bf16* __restrict__ A,
                           __bf16* __restrict__ AT) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * N) return;
  const long m = i / N;
  const int n = (int)(i - m * N);
  const __bf16 a = (__bf16)gelu(Z[i]);
  A[i] = a;
  if (AT) AT[(long)n * M + m] = a;
}

// dZ = dA * gelu'(Z): bf16 row-major and transposed, and fp32 row-major
__global__ void k_gelu_bwd(const float* __restrict__ dA, const float* __restrict__ Z, long M, int N,
                           __bf16* __restrict__ dZ, __bf16* __restrict__ dZT, float* __restrict__ dZf) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M * N) return;
  const long m = i / N;
  const int n = (int)(i - m * N);
  const float d = dA[i] * gelu_d(Z[i]);
  dZ[i] = (__bf16)d;
  dZT[(long)n * M + m] = (__bf16)d;
  dZf[i] = d;
}

// sum of `parts` arrays of length n
__global__ void k_sum_parts(const float* __restrict__ p, int parts, long n, float* __restrict__ out) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = 0.f;
  for (int q = 0; q < parts; ++q) s += p[(long)q * n + i];
  out[i] = s;
}

// column sums of X[M x N] (fp32): out[n] = sum_m X[m][n]
__global__ void k_colsum(const float* __restrict__ X, long M, int N, float* __restrict__ out) {
  const int n = blockIdx.x;
  float s = 0.f;
  for (long m = threadIdx.x; m < M; m += blockDim.x) s += X[m * N + n];
  __shared__ float red[256];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d) red[threadIdx.x] += red[threadIdx.x + d];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[n] = red[0];
}

// Head (256 -> 2, fp32) on bf16 activations: out = A W^T + b
__global__ void k_head_fwd(const __bf16* __restrict__ A, const float* __restrict__ W, const float* __restrict__ b,
                           long M, float* __restrict__ out) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  float s0 = b[0], s1 = b[1];
  const __bf16* a = A + m * 256;
  for (int k = 0; k < 256; ++k) {
    const float v = (float)a[k];
    s0 = fmaf(v, W[k], s0);
    s1 = fmaf(v, W[256 + k], s1);
  }
  out[2 * m] = s0;
  out[2 * m + 1] = s1;
}

// Loss 0.5 mean_m |out - y|^2 (sum over the 2 outputs): dOut = (out - y) / M;
// dA = dOut W (fp32 [M x 256]); per-block partial sums of the loss, dW, db.
__global__ __launch_bounds__(256) void k_head_bwd(const __bf16* __restrict__ A, const float* __restrict__ W,
                                                  const float* __restrict__ out, const float* __restrict__ y,
                                                  long M, float* __restrict__ dA, float* __restrict__ part) {
  // part layout per block: [loss, db0, db1, dW (2 x 256)]
  __shared__ float red[256][4];
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  float d0 = 0.f, d1 = 0.f, l = 0.f;
  if (m < M) {
    const float e0 = out[2 * m] - y[2 * m], e1 = out[2 * m + 1] - y[2 * m + 1];
    l = 0.5f * (e0 * e0 + e1 * e1) / (float)M;
    d0 = e0 / (float)M;
    d1 = e1 / (float)M;
    for (int k = 0; k < 256; ++k) dA[m * 256 + k] = d0 * W[k] + d1 * W[256 + k];
  }
  red[threadIdx.x][0] = l;
  red[threadIdx.x][1] = d0;
  red[threadIdx.x][2] = d1;
  __syncthreads();
  for (int d = 128; d > 0; d >>= 1) {
    if ((int)threadIdx.x < d)
      for (int c = 0; c < 3; ++c) red[threadIdx.x][c] += red[threadIdx.x + d][c];
    __syncthreads();
  }
  float* P = part + (long)blockIdx.x * (3 + 512);
  if (threadIdx.x == 0) {
    P[0] = red[0][0];
    P[1] = red[0][1];
    P[2] = red[0][2];
  }
  // dW[o][k] = sum_m dOut[m][o] A[m][k]: thread k accumulates over the block's rows
  __shared__ float dsh[256][2];
  dsh[threadIdx.x][0] = d0;
  dsh[threadIdx.x][1] = d1;
  __syncthreads();
  const int k = threadIdx.x;
  float w0 = 0.f, w1 = 0.f;
  const long mb = (long)blockIdx.x * blockDim.x;
  for (int r = 0; r < 256 && mb + r < M; ++r) {
    const float a = (float)A[(mb + r) * 256 + k];
    w0 = fmaf(dsh[r][0], a, w0);
    w1 = fmaf(dsh[r][1], a, w1);
  }
  P[3 + k] = w0;
  P[3 + 256 + k] = w1;
}

// Adam on fp32 parameters; bf16 copies (row-major and transposed) of the
// hidden weight matrices are refreshed by k_refresh_bf16.
__global__ void k_adam(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m1,
                       float* __restrict__ m2, long n, float lr, float b1, float b2, float eps, float c1, float c2) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float a = b1 * m1[i] + (1.f - b1) * gi;
  const float b = b2 * m2[i] + (1.f - b2) * gi * gi;
  m1[i] = a;
  m2[i] = b;
  p[i] -= lr * (a / c1) / (sqrtf(b / c2) + eps);
}

__global__ void k_refresh_bf16(const float* __restrict__ W, int N, int K, __bf16* __restrict__ Wb,
                               __bf16* __restrict__ WTb) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)N * K) return;
  const int n = (int)(i / K), k = (int)(i - (long)n * K);
  const __bf16 v = (__bf16)W[i];
  Wb[i] = v;
  if (WTb) WTb[(long)k * N + n] = v;
}

// The 64 input features of one query (x1, x2, x3, k, alpha1, alpha2).
__device__ __forceinline__ void features_row(const double* __restrict__ Q, double c, double c_tilde, float f[64]) {
  const double x1 = Q[0], x2 = Q[1], x3 = Q[2], k = Q[3], a1 = Q[4], a2 = Q[5];
  const double t1 = x1 - 2.0 * kPi * floor((x1 + kPi) * (0.5 / kPi));
  const double t2 = x2 - 2.0 * kPi * floor((x2 + kPi) * (0.5 / kPi));
  int o = 0;
  // harmonics h = 1 .. nh of an angle: one sine and cosine, then rotations by it (FP64, so the
  // recurrence's rounding stays far below the features' bf16 precision)
  auto harmonics = [&](double th, int nh) {
    double s1, c1;
    sincos(th, &s1, &c1);
    double cs = c1, sn = s1;
    for (int h = 1; h <= nh; ++h) {
      f[o++] = (float)cs;
      f[o++] = (float)sn;
      const double cn = cs * c1 - sn * s1;
      sn = sn * c1 + cs * s1;
      cs = cn;
    }
  };
  harmonics(t1, 8);
  harmonics(t2, 8);
  const double z = kPi * x3 / c_tilde;
  harmonics(z, 6);
  const double r = sqrt(t1 * t1 + t2 * t2 + x3 * x3);
  f[o++] = (float)(x3 / c);
  f[o++] = (float)((k - 5.5) / 4.5);
  f[o++] = (float)(2.0 * a1);
  f[o++] = (float)(2.0 * a2);
  const double args[8] = {k * t1, k * t2, k * x3, k * r, a1 * t1, a2 * t2, 2.0 * kPi * a1, 2.0 * kPi * a2};
  for (int h = 0; h < 8; ++h) {
    double sn, cs;
    sincos(args[h], &sn, &cs);
    f[o++] = (float)cs;
    f[o++] = (float)sn;
  }
}

// Features of M queries in bf16, row-major, and optionally transposed.
__global__ void k_features(const double* __restrict__ q, long M, double c, double c_tilde, __bf16* __restrict__ F,
                           __bf16* __restrict__ FT) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  float f[64];
  features_row(q + 6 * m, c, c_tilde, f);
  for (int h = 0; h < 64; ++h) {
    const __bf16 v = (__bf16)f[h];
    F[m * 64 + h] = v;
    if (FT) FT[(long)h * M + m] = v;
  }
}

// ---------------------------------------------------------------------------
// Fused inference: one block takes kIR queries through every ensemble member.
// Features, then four hidden layers with the activations of the tile held in
// LDS (two ping-pong buffers), weights read from L2, the K = 32 bf16 matrix
// instruction, bias + GELU in the epilogue, and the fp32 head.  Four waves; wave w computes output columns
// [64 w, 64 w + 64) of a hidden layer for all rows of the tile (16 x 16 tiles).
// The rounding points are those of the layer-by-layer path: bf16 features,
// fp32 accumulation plus fp32 bias, GELU in fp32, bf16 activations.
// ---------------------------------------------------------------------------
constexpr int kIR = 128;                 // rows per block
constexpr int kIP0 = 64 + 8, kIP = 256 + 8;   // LDS row pitches (bf16) of features / activations
constexpr int kMaxMembers = 8;

struct InferArgs {
  const __bf16* wb[kMaxMembers];   // hidden weights [4][256][K] (K = 64 for layer 0, 256 after)
  const float* p[kMaxMembers];     // fp32 parameters: biases and the head
  long off_b[4], off_w4, off_b4;   // offsets in p
  int members;
  double c, c_tilde;
};


// erf by Abramowitz & Stegun 7.1.26 (|error| <= 1.5e-7, far below the bf16 rounding of the
// activations it feeds): the inference kernel's GELU
__device__ __forceinline__ float erf_as(float x) {
  const float ax = fabsf(x);
  const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, ax, 1.0f));
  const float p = t * fmaf(t, fmaf(t, fmaf(t, fmaf(t, 1.061405429f, -1.453152027f), 1.421413741f), -0.284496736f),
                           0.254829592f);
  return copysignf(1.0f - p * __expf(-ax * ax), x);
}
__device__ __forceinline__ float gelu_inf(float z) { return 0.5f * z * (1.f + erf_as(z * 0.70710678118654752f)); }

template <int K>
__device__ __forceinline__ void infer_layer(const __bf16* __restrict__ X, int pitchX, const __bf16* __restrict__ W,
                                            const float* __restrict__ bias, __bf16* __restrict__ Y) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int lr = lane & 15, lg = lane >> 4;
  constexpr int RT = kIR / 16;   // row tiles of 16
  f32x4 acc[RT][4];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  // v_mfma_f32_16x16x32_bf16: lane l holds A[l % 16][8 (l / 16) + r] and
  // B[8 (l / 16) + r][l % 16], r < 8 (16-byte fragments)
  for (int k0 = 0; k0 < K; k0 += 32) {
    bf16x8 b[4];
#pragma unroll
    for (int j = 0; j < 4; ++j)
      b[j] = *reinterpret_cast<const bf16x8*>(W + (long)(64 * w + 16 * j + lr) * K + k0 + 8 * lg);
#pragma unroll
    for (int i = 0; i < RT; ++i) {
      const bf16x8 a = *reinterpret_cast<const bf16x8*>(X + (16 * i + lr) * pitchX + k0 + 8 * lg);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b[j], acc[i][j], 0, 0, 0);
    }
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int col = 64 * w + 16 * j + lr;
    const float bb = bias[col];
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int r = 0; r < 4; ++r) Y[(16 * i + 4 * lg + r) * kIP + col] = (__bf16)gelu_inf(acc[i][j][r] + bb);
  }
}

__global__ __launch_bounds__(256) void k_mlp_infer(InferArgs A, const double* __restrict__ q, long M,
                                                   float* __restrict__ y, long ystride) {
  __shared__ __bf16 X0[kIR * kIP0];
  __shared__ __bf16 B1[kIR * kIP];
  __shared__ __bf16 B2[kIR * kIP];
  const long r0 = (long)blockIdx.x * kIR;
  if (threadIdx.x < kIR) {
    const long m = r0 + threadIdx.x;
    float f[64];
    if (m < M) features_row(q + 6 * m, A.c, A.c_tilde, f);
    else
      for (int h = 0; h < 64; ++h) f[h] = 0.f;
    for (int h = 0; h < 64; ++h) X0[threadIdx.x * kIP0 + h] = (__bf16)f[h];
  }
  __syncthreads();
  for (int e = 0; e < A.members; ++e) {
    const __bf16* wb = A.wb[e];
    const float* p = A.p[e];
    infer_layer<64>(X0, kIP0, wb, p + A.off_b[0], B1);
    __syncthreads();
    infer_layer<256>(B1, kIP, wb + 256 * 256, p + A.off_b[1], B2);
    __syncthreads();
    infer_layer<256>(B2, kIP, wb + 2 * 256 * 256, p + A.off_b[2], B1);
    __syncthreads();
    infer_layer<256>(B1, kIP, wb + 3 * 256 * 256, p + A.off_b[3], B2);
    __syncthreads();
    // head: thread t -> row t / 2, output t % 2
    if (threadIdx.x < 2 * kIR) {
      const int row = threadIdx.x >> 1, o = threadIdx.x & 1;
      const float* W4 = p + A.off_w4 + o * 256;
      float s_ = p[A.off_b4 + o];
      const __bf16* a = B2 + row * kIP;
      for (int k = 0; k < 256; ++k) s_ = fmaf((float)a[k], W4[k], s_);
      const long m = r0 + row;
      if (m < M) y[(long)e * ystride + 2 * m + o] = s_;
    }
    __syncthreads();
  }
}

// Queries of many instances: q[m] = (x[m], k_i, a1_i, a2_i) for t0_i <= m < t1_i.
struct QInst {
  double k, a1, a2;
  long t0, t1;
};
__global__ void k_make_queries(const QInst* __restrict__ inst, int n, const double* __restrict__ x, long T,
                               double* __restrict__ q) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= T) return;
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].t0 <= m) lo = mid;
    else hi = mid - 1;
  }
  const QInst I = inst[lo];
  double* Q = q + 6 * m;
  Q[0] = x[3 * m];
  Q[1] = x[3 * m + 1];
  Q[2] = x[3 * m + 2];
  Q[3] = I.k;
  Q[4] = I.a1;
  Q[5] = I.a2;
}

// Distance to a Wood anomaly: min over lattice points of |k^2 - |alpha + n|^2|^{1/2}.
__device__ double wood_distance(double k, double a1, double a2) {
  double best = 1e300;
  const int n1lo = (int)floor(-k - a1) - 1, n1hi = (int)ceil(k - a1) + 1;
  for (int n1 = n1lo; n1 <= n1hi; ++n1) {
    const double e1 = a1 + n1;
    const double r2 = k * k - e1 * e1;
    const double c = r2 > 0.0 ? sqrt(r2) : 0.0;
    const double cand[4] = {floor(c - a2), ceil(c - a2), floor(-c - a2), ceil(-c - a2)};
    for (int j = 0; j < 4; ++j) {
      const double e2 = a2 + cand[j];
      best = fmin(best, sqrt(fabs(k * k - e1 * e1 - e2 * e2)));
    }
  }
  return best;
}

// Ensemble mean of L_d (the outputs are 10 L_d) and its spread: the largest distance of a member
// from the mean.
__device__ inline void ensemble_stats(const float* __restrict__ y, int members, long ystride, long m, double& mr,
                                      double& mi, double& spread) {
  mr = 0.0;
  mi = 0.0;
  for (int e = 0; e < members; ++e) {
    mr += y[e * ystride + 2 * m];
    mi += y[e * ystride + 2 * m + 1];
  }
  mr /= members;
  mi /= members;
  spread = 0.0;
  for (int e = 0; e < members; ++e) {
    const double dr = y[e * ystride + 2 * m] - mr, di = y[e * ystride + 2 * m + 1] - mi;
    spread = fmax(spread, sqrt(dr * dr + di * di));
  }
  mr *= 0.1;
  mi *= 0.1;
  spread *= 0.1;
}

// Combine the ensemble into G_d with the FP64 add-back, and decide fallback: far branch, Wood
// anomaly, lattice proximity, or an error estimate kappa * spread above tol |G_d|.  kappa comes from
// calibration against the plain method; it is +inf until then (and the estimate is not formed with
// fewer than two members), so an uncalibrated model accepts nothing.
template <typename T>
__global__ void k_surrogate_combine(const double* __restrict__ q, long M, const float* __restrict__ y, int members,
                                    long ystride, double c, double eps, double tol, double kappa, double wood_tol,
                                    double rmin, cplx<T>* __restrict__ out, uint8_t* __restrict__ fell) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  const double* Q = q + 6 * m;
  const double x1 = Q[0], x2 = Q[1], x3 = Q[2], k = Q[3], a1 = Q[4], a2 = Q[5];
  double n1 = floor((x1 + kPi) * (0.5 / kPi)), n2 = floor((x2 + kPi) * (0.5 / kPi));
  const double t1 = x1 - 2.0 * kPi * n1, t2 = x2 - 2.0 * kPi * n2;
  double mr, mi, spread;
  ensemble_stats(y, members, ystride, m, mr, mi, spread);
  const double2 L = mk(mr, mi);
  const double r = sqrt(t1 * t1 + t2 * t2 + x3 * x3);
  double ps, pc;
  sincos(a1 * x1 + a2 * x2, &ps, &pc);
  double2 G = cmul(mk(pc, ps), L);
  if (r < 2.0 * eps && r > 0.0) {
    double sn, cn;
    sincos(k * r, &sn, &cn);
    double ls, lc;
    sincospi(2.0 * (a1 * n1 + a2 * n2), &ls, &lc);
    const double s = cut_Y(r, eps) / (4.0 * kPi * r);
    G = cadd(G, cmul(mk(lc, ls), mk(cn * s, sn * s)));
  }
  uint8_t fb = 0;
  if (!(fabs(x3) <= c)) fb |= 2;
  if (!(members >= 2 && kappa * spread <= tol * sqrt(G.x * G.x + G.y * G.y))) fb |= 4;
  if (wood_distance(k, a1, a2) < wood_tol) fb |= 8;
  if (r <= rmin) fb |= 16;
  cplx<T> v;
  v.x = (T)G.x;
  v.y = (T)G.y;
  out[m] = v;
  fell[m] = fb;
}

// Calibration: ratio[m] = |L_mean - L| / spread against the plain method's smooth part L (NaN where
// L is NaN, i.e. far targets; +inf where the members agree exactly but the mean is off).
template <typename T>
__global__ void k_calib_ratio(long M, const float* __restrict__ y, int members, long ystride,
                              const cplx<T>* __restrict__ Lp, double* __restrict__ ratio) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= M) return;
  double mr, mi, spread;
  ensemble_stats(y, members, ystride, m, mr, mi, spread);
  const cplx<T> l = Lp[m];
  const double dr = mr - (double)l.x, di = mi - (double)l.y;
  const double err = sqrt(dr * dr + di * di);
  ratio[m] = err != err ? err : (spread > 0.0 ? err / spread : (err > 0.0 ? __builtin_inf() : 0.0));
}

// Training rows of one instance: q = (x, k, alpha1, alpha2), y = 10 L (float32).
template <typename T>
__global__ void k_make_rows(const double* __restrict__ x, long n, double k, double a1, double a2,
                            const cplx<T>* __restrict__ Lp, double* __restrict__ q, float* __restrict__ y) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= n) return;
  double* Q = q + 6 * m;
  Q[0] = x[3 * m];
  Q[1] = x[3 * m + 1];
  Q[2] = x[3 * m + 2];
  Q[3] = k;
  Q[4] = a1;
  Q[5] = a2;
  const cplx<T> l = Lp[m];
  y[2 * m] = (float)(10.0 * (double)l.x);
  y[2 * m + 1] = (float)(10.0 * (double)l.y);
}

// One minibatch: rows idx[0..B) of (q, y) side by side.
__global__ void k_gather_rows(const double* __restrict__ q, const float* __restrict__ y,
                              const uint32_t* __restrict__ idx, long B, double* __restrict__ qb,
                              float* __restrict__ yb) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= B) return;
  const long r = idx[m];
  for (int j = 0; j < 6; ++j) qb[6 * m + j] = q[6 * r + j];
  yb[2 * m] = y[2 * r];
  yb[2 * m + 1] = y[2 * r + 1];
}

}  // namespace

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
hipError_t mlp_gemm(hipStream_t st, const __bf16* A, long a_m, long a_k, const __bf16* B, long b_k, long b_n,
                    float* C, long c_m, long c_n, const float* bias, int M, int N, int K, int splits) {
  GemmArgs g;
  g.A = A;
  g.a_m = a_m;
  g.a_k = a_k;
  g.B = B;
  g.b_k = b_k;
  g.b_n = b_n;
  g.C = C;
  g.c_m = c_m;
  g.c_n = c_n;
  g.c_split = (long)M * N;
  g.bias = bias;
  g.M = M;
  g.N = N;
  g.K = K;
  g.ksplit = ((K / splits + 15) / 16) * 16;
  hipLaunchKernelGGL(k_gemm_bf16, dim3(N / 64, M / 64, splits), dim3(256), 0, st, g);
  return hipGetLastError();
}

static unsigned nb(long n, int b = 256) { return (unsigned)((n + b - 1) / b); }

hipError_t mlp_gelu_fwd(hipStream_t st, const float* Z, long M, int N, __bf16* A, __bf16* AT) {
  hipLaunchKernelGGL(k_gelu_fwd, dim3(nb(M * N)), dim3(256), 0, st, Z, M, N, A, AT);
  return hipGetLastError();
}
hipError_t mlp_gelu_bwd(hipStream_t st, const float* dA, const float* Z, long M, int N, __bf16* dZ, __bf16* dZT,
                        float* dZf) {
  hipLaunchKernelGGL(k_gelu_bwd, dim3(nb(M * N)), dim3(256), 0, st, dA, Z, M, N, dZ, dZT, dZf);
  return hipGetLastError();
}
hipError_t mlp_sum_parts(hipStream_t st, const float* p, int parts, long n, float* out) {
  hipLaunchKernelGGL(k_sum_parts, dim3(nb(n)), dim3(256), 0, st, p, parts, n, out);
  return hipGetLastError();
}
hipError_t mlp_colsum(hipStream_t st, const float* X, long M, int N, float* out) {
  hipLaunchKernelGGL(k_colsum, dim3(N), dim3(256), 0, st, X, M, N, out);
  return hipGetLastError();
}
hipError_t mlp_head_fwd(hipStream_t st, const __bf16* A, const float* W, const float* b, long M, float* out) {
  hipLaunchKernelGGL(k_head_fwd, dim3(nb(M)), dim3(256), 0, st, A, W, b, M, out);
  return hipGetLastError();
}
hipError_t mlp_head_bwd(hipStream_t st, const __bf16* A, const float* W, const float* out, const float* y, long M,
                        float* dA, float* part) {
  hipLaunchKernelGGL(k_head_bwd, dim3(nb(M)), dim3(256), 0, st, A, W, out, y, M, dA, part);
  return hipGetLastError();
}
hipError_t mlp_adam(hipStream_t st, float* p, const float* g, float* m1, float* m2, long n, float lr, float b1,
                    float b2, float eps, float c1, float c2) {
  hipLaunchKernelGGL(k_adam, dim3(nb(n)), dim3(256), 0, st, p, g, m1, m2, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}
hipError_t mlp_refresh_bf16(hipStream_t st, const float* W, int N, int K, __bf16* Wb, __bf16* WTb) {
  hipLaunchKernelGGL(k_refresh_bf16, dim3(nb((long)N * K)), dim3(256), 0, st, W, N, K, Wb, WTb);
  return hipGetLastError();
}
hipError_t mlp_features(hipStream_t st, const double* q, long M, double c, double c_tilde, __bf16* F, __bf16* FT) {
  hipLaunchKernelGGL(k_features, dim3(nb(M)), dim3(256), 0, st, q, M, c, c_tilde, F, FT);
  return hipGetLastError();
}
hipError_t mlp_infer(hipStream_t st, const __bf16* const* wb, const float* const* p, int members, const long off_b[4],
                     long off_w4, long off_b4, double c, double c_tilde, const double* q, long M, float* y,
                     long ystride) {
  if (members < 1 || members > kMaxMembers) return hipErrorInvalidValue;
  InferArgs A;
  for (int e = 0; e < kMaxMembers; ++e) {
    A.wb[e] = e < members ? wb[e] : nullptr;
    A.p[e] = e < members ? p[e] : nullptr;
  }
  for (int l = 0; l < 4; ++l) A.off_b[l] = off_b[l];
  A.off_w4 = off_w4;
  A.off_b4 = off_b4;
  A.members = members;
  A.c = c;
  A.c_tilde = c_tilde;
  hipLaunchKernelGGL(k_mlp_infer, dim3((unsigned)((M + kIR - 1) / kIR)), dim3(256), 0, st, A, q, M, y, ystride);
  return hipGetLastError();
}
size_t mlp_qinst_size() { return sizeof(QInst); }
size_t mlp_qinst_t0_offset() { return offsetof(QInst, t0); }
void mlp_qinst(double k, double a1, double a2, long t0, long t1, void* dst) {
  QInst I{k, a1, a2, t0, t1};
  *static_cast<QInst*>(dst) = I;
}
hipError_t mlp_make_queries(hipStream_t st, const void* inst, int n, const double* x, long T, double* q) {
  hipLaunchKernelGGL(k_make_queries, dim3(nb(T)), dim3(256), 0, st, static_cast<const QInst*>(inst), n, x, T, q);
  return hipGetLastError();
}
hipError_t mlp_combine(hipStream_t st, int prec, const double* q, long M, const float* y, int members, long ystride,
                       double c, double eps, double tol, double kappa, double wood_tol, double rmin, void* out,
                       uint8_t* fell) {
  if (prec == QPGF_C128)
    hipLaunchKernelGGL(k_surrogate_combine<double>, dim3(nb(M)), dim3(256), 0, st, q, M, y, members, ystride, c, eps,
                       tol, kappa, wood_tol, rmin, static_cast<double2*>(out), fell);
  else
    hipLaunchKernelGGL(k_surrogate_combine<float>, dim3(nb(M)), dim3(256), 0, st, q, M, y, members, ystride, c, eps,
                       tol, kappa, wood_tol, rmin, static_cast<float2*>(out), fell);
  return hipGetLastError();
}
hipError_t mlp_calib_ratio(hipStream_t st, int prec, long M, const float* y, int members, long ystride, const void* L,
                           double* ratio) {
  if (prec == QPGF_C128)
    hipLaunchKernelGGL(k_calib_ratio<double>, dim3(nb(M)), dim3(256), 0, st, M, y, members, ystride,
                       static_cast<const double2*>(L), ratio);
  else
    hipLaunchKernelGGL(k_calib_ratio<float>, dim3(nb(M)), dim3(256), 0, st, M, y, members, ystride,
                       static_cast<const float2*>(L), ratio);
  return hipGetLastError();
}
hipError_t mlp_make_rows(hipStream_t st, int prec, const double* x, long n, double k, double a1, double a2,
                         const void* L, double* q, float* y) {
  if (prec == QPGF_C128)
    hipLaunchKernelGGL(k_make_rows<double>, dim3(nb(n)), dim3(256), 0, st, x, n, k, a1, a2,
                       static_cast<const double2*>(L), q, y);
  else
    hipLaunchKernelGGL(k_make_rows<float>, dim3(nb(n)), dim3(256), 0, st, x, n, k, a1, a2,
                       static_cast<const float2*>(L), q, y);
  return hipGetLastError();
}
hipError_t mlp_gather_rows(hipStream_t st, const double* q, const float* y, const uint32_t* idx, long B, double* qb,
                           float* yb) {
  hipLaunchKernelGGL(k_gather_rows, dim3(nb(B)), dim3(256), 0, st, q, y, idx, B, qb, yb);
  return hipGetLastError();
}

}  // namespace qpgf
