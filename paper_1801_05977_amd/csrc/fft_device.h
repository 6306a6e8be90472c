// Device building blocks of the inverse DFTs (unnormalised, e^{+2 pi i jp/n},
// lengths n = 2^a r with r in {1, 3, 5, 7}): radix-8/4/2 and radix-3/5/7
// butterflies in registers and one in-place Stockham autosort pass over
// transforms held in LDS.  Shared by the FFT kernels and by the 3D fill, which
// transforms its pencils along the transverse axis before writing them.
#pragma once

#include "qpgf_internal.h"

namespace qpgf {

// A block of `tile` transforms of length n (row pitch `pitch`) also holds the n
// twiddles of that length in LDS when both fit in 64 KiB; otherwise the passes
// read the plan's twiddle table from global memory.
__host__ __device__ inline bool fft_twiddles_in_lds(long tile, int pitch, int n, size_t esize) {
  return ((size_t)tile * pitch + (size_t)n) * esize <= 65536;
}

namespace fftdev {

template <typename V> __device__ __forceinline__ V c_add(V a, V b) { V r; r.x = a.x + b.x; r.y = a.y + b.y; return r; }
template <typename V> __device__ __forceinline__ V c_sub(V a, V b) { V r; r.x = a.x - b.x; r.y = a.y - b.y; return r; }
template <typename V> __device__ __forceinline__ V c_mul(V a, V b) {
  V r;
  r.x = a.x * b.x - a.y * b.y;
  r.y = a.x * b.y + a.y * b.x;
  return r;
}
// a + i b, a - i b
template <typename V> __device__ __forceinline__ V c_addi(V a, V b) { V r; r.x = a.x - b.y; r.y = a.y + b.x; return r; }
template <typename V> __device__ __forceinline__ V c_subi(V a, V b) { V r; r.x = a.x + b.y; r.y = a.y - b.x; return r; }

// inverse radix-8 DFT in registers: y_m = sum_r v_r e^{+2 pi i r m / 8}
template <typename V, typename T>
__device__ __forceinline__ void dft8(V v[8]) {
  const T h = (T)0.70710678118654752440;
  const V a0 = c_add(v[0], v[4]), a1 = c_sub(v[0], v[4]), a2 = c_add(v[2], v[6]), a3 = c_sub(v[2], v[6]);
  const V a4 = c_add(v[1], v[5]), a5 = c_sub(v[1], v[5]), a6 = c_add(v[3], v[7]), a7 = c_sub(v[3], v[7]);
  const V e0 = c_add(a0, a2), e2 = c_sub(a0, a2), e1 = c_addi(a1, a3), e3 = c_subi(a1, a3);
  const V o0 = c_add(a4, a6), o2 = c_sub(a4, a6), o1 = c_addi(a5, a7), o3 = c_subi(a5, a7);
  // w^1 o1 = (1 + i)/sqrt2 o1, w^2 o2 = i o2, w^3 o3 = (-1 + i)/sqrt2 o3
  V w1, w3;
  w1.x = h * (o1.x - o1.y);
  w1.y = h * (o1.x + o1.y);
  w3.x = -h * (o3.x + o3.y);
  w3.y = h * (o3.x - o3.y);
  v[0] = c_add(e0, o0);
  v[4] = c_sub(e0, o0);
  v[1] = c_add(e1, w1);
  v[5] = c_sub(e1, w1);
  v[2] = c_addi(e2, o2);
  v[6] = c_subi(e2, o2);
  v[3] = c_add(e3, w3);
  v[7] = c_sub(e3, w3);
}

template <typename V>
__device__ __forceinline__ void dft4(V v[4]) {
  const V a0 = c_add(v[0], v[2]), a1 = c_sub(v[0], v[2]), a2 = c_add(v[1], v[3]), a3 = c_sub(v[1], v[3]);
  v[0] = c_add(a0, a2);
  v[1] = c_addi(a1, a3);
  v[2] = c_sub(a0, a2);
  v[3] = c_subi(a1, a3);
}

template <typename V>
__device__ __forceinline__ void dft2(V v[2]) {
  const V a = v[0];
  v[0] = c_add(a, v[1]);
  v[1] = c_sub(a, v[1]);
}

// cos and sin of 2 pi q / R for the odd radices (q = 1 .. (R - 1)/2)
__host__ __device__ constexpr double cos_odd(int R, int q) {
  return R == 3 ? -0.5
         : R == 5 ? (q == 1 ? 0.30901699437494742410 : -0.80901699437494742410)
                  : (q == 1 ? 0.62348980185873353053 : q == 2 ? -0.22252093395631440429 : -0.90096886790241912624);
}
__host__ __device__ constexpr double sin_odd(int R, int q) {
  return R == 3 ? 0.86602540378443864676
         : R == 5 ? (q == 1 ? 0.95105651629515357212 : 0.58778525229247312917)
                  : (q == 1 ? 0.78183148246802980871 : q == 2 ? 0.97492791218182360702 : 0.43388373911755812048);
}

// inverse DFT of odd prime length R in registers, y_m = sum_r v_r e^{+2 pi i r m / R}: the inputs
// r and R - r share cos(2 pi r m / R) and carry opposite sines, so each pair of outputs m, R - m
// takes (R - 1)/2 cosine and sine sums over a_q = v_q + v_{R-q} and b_q = v_q - v_{R-q}
template <int R, typename V, typename T>
__device__ __forceinline__ void dft_odd(V v[R]) {
  constexpr int H = (R - 1) / 2;
  V a[H], b[H];
#pragma unroll
  for (int q = 1; q <= H; ++q) {
    a[q - 1] = c_add(v[q], v[R - q]);
    b[q - 1] = c_sub(v[q], v[R - q]);
  }
  V out[R];
  out[0] = v[0];
#pragma unroll
  for (int q = 0; q < H; ++q) out[0] = c_add(out[0], a[q]);
#pragma unroll
  for (int m = 1; m <= H; ++m) {
    V cr = v[0], si;
    si.x = 0;
    si.y = 0;
#pragma unroll
    for (int q = 1; q <= H; ++q) {
      const int qm = (q * m) % R;                     // cos(2 pi qm / R) = cos(2 pi id / R)
      const int id = qm <= H ? qm : R - qm;
      const T c = (T)cos_odd(R, id);
      const T sn = (T)(qm <= H ? sin_odd(R, id) : -sin_odd(R, id));
      cr.x += c * a[q - 1].x;
      cr.y += c * a[q - 1].y;
      si.x += sn * b[q - 1].x;
      si.y += sn * b[q - 1].y;
    }
    out[m] = c_addi(cr, si);       // y_m = cr + i si
    out[R - m] = c_subi(cr, si);   // y_{R-m} = cr - i si
  }
#pragma unroll
  for (int r = 0; r < R; ++r) v[r] = out[r];
}

template <int R, typename V, typename T>
__device__ __forceinline__ void dftR(V v[R]) {
  if constexpr (R == 8) dft8<V, T>(v);
  else if constexpr (R == 4) dft4<V>(v);
  else if constexpr (R == 2) dft2<V>(v);
  else dft_odd<R, V, T>(v);
}

// One in-place Stockham pass of radix R over `ntile` transforms of length n
// held in LDS (row pitch `pitch`): every thread first reads its butterflies'
// inputs into registers, the block synchronises, then writes the outputs.
// Ns (the product of the radices already applied) is a power of two: the odd
// radix, if any, takes the last pass.  Twiddles e^{2 pi i q / ntw} at stride
// ntw / (Ns R) from a table of ntw entries.  At most MAXB butterflies per thread
// (256 threads).
template <typename T, int R, int MAXB>
__device__ __forceinline__ void stockham_pass(cplx<T>* buf, int n, int pitch, int ntile, int Ns,
                                              const cplx<T>* __restrict__ tw, int ntw) {
  using V = cplx<T>;
  const int nb = n / R;
  const int total = ntile * nb;
  const int step = ntw / (Ns * R);
  V v[MAXB][R];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int idx = threadIdx.x + q * 256;
    if (idx < total) {
      const int t = idx / nb, j = idx - t * nb;
      const V* src = buf + t * pitch + j;
#pragma unroll
      for (int r = 0; r < R; ++r) v[q][r] = src[r * nb];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int idx = threadIdx.x + q * 256;
    if (idx < total) {
      const int t = idx / nb, j = idx - t * nb;
      const int kk = j & (Ns - 1);
      if (Ns > 1) {
#pragma unroll
        for (int r = 1; r < R; ++r) v[q][r] = c_mul(v[q][r], tw[(r * kk) * step]);
      }
      dftR<R, V, T>(v[q]);
      V* dst = buf + t * pitch + (j - kk) * R + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[q][r];
    }
  }
  __syncthreads();
}

// LDS capacity of one block, in complex elements (64 KiB).
template <typename T> constexpr int lds_cap() { return 65536 / (int)sizeof(cplx<T>); }


// All passes of inverse DFTs of length n = 2^a r (r in {1, 3, 5, 7}) over `ntile` transforms in
// LDS (row pitch `pitch`): radix-8 passes, one radix-4 or radix-2 pass for the rest of 2^a, then
// the radix-r pass.  256 threads; ntile * n <= lds_cap<T>(); tw holds ntw twiddles, n | ntw.
template <typename T>
__device__ __forceinline__ void inverse_dft_lds(cplx<T>* buf, int n, int pitch, int ntile,
                                                const cplx<T>* __restrict__ tw, int ntw) {
  constexpr int CAP = lds_cap<T>();
  const int odd = n >> __builtin_ctz((unsigned)n);
  int Ns = 1, rem = __builtin_ctz((unsigned)n);
  while (rem >= 3) {
    stockham_pass<T, 8, CAP / (8 * 256)>(buf, n, pitch, ntile, Ns, tw, ntw);
    Ns <<= 3;
    rem -= 3;
  }
  if (rem == 2) stockham_pass<T, 4, CAP / (4 * 256)>(buf, n, pitch, ntile, Ns, tw, ntw);
  else if (rem == 1) stockham_pass<T, 2, CAP / (2 * 256)>(buf, n, pitch, ntile, Ns, tw, ntw);
  Ns <<= rem;
  if (odd == 3) stockham_pass<T, 3, (CAP + 3 * 256 - 1) / (3 * 256)>(buf, n, pitch, ntile, Ns, tw, ntw);
  else if (odd == 5) stockham_pass<T, 5, (CAP + 5 * 256 - 1) / (5 * 256)>(buf, n, pitch, ntile, Ns, tw, ntw);
  else if (odd == 7) stockham_pass<T, 7, (CAP + 7 * 256 - 1) / (7 * 256)>(buf, n, pitch, ntile, Ns, tw, ntw);
}

// Lengths the transforms take: 2^a r, r in {1, 3, 5, 7} (r = 1: powers of two).
__host__ __device__ inline bool fft_length_ok(int n) {
  if (n < 2) return false;
  const int odd = n >> __builtin_ctz((unsigned)n);
  return odd == 1 || odd == 3 || odd == 5 || odd == 7;
}

}  // namespace fftdev
}  // namespace qpgf
