// Batched inverse DFTs (unnormalised, e^{+2 pi i jp/n}) along one axis of a
// strided array: the grid synthesis of Algorithms 2.1 / 3.1 / 4.1 (steps 1c-1d),
// L_N(x_p) = sum_j L-hat_j e^{i pi j p / N}, with coefficients and grid points
// both stored mod n.  Power-of-two lengths, radix-4 (plus one radix-2) Stockham
// autosort passes staged in LDS.
//
// Batch b of a launch starts at element (b / b_in) * s_out + (b % b_in) * s_in
// and its elements are elem_stride apart.  A block takes `tile` consecutive
// batches: for rows (elem_stride 1) each batch is one contiguous run, for
// columns (s_in 1) the tile's batches are adjacent, so both load coalesced.
#include <algorithm>

#include "qpgf_internal.h"

namespace qpgf {

namespace {

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

template <int R, typename V, typename T>
__device__ __forceinline__ void dftR(V v[R]) {
  if constexpr (R == 8) dft8<V, T>(v);
  else if constexpr (R == 4) dft4<V>(v);
  else dft2<V>(v);
}

// One in-place Stockham pass of radix R over `ntile` transforms of length n
// held in LDS (row pitch `pitch`): every thread first reads its butterflies'
// inputs into registers, the block synchronises, then writes the outputs.
// At most MAXB butterflies per thread (256 threads).
template <typename T, int R, int MAXB>
__device__ __forceinline__ void stockham_pass(cplx<T>* buf, int n, int pitch, int ntile, int Ns, int lr,
                                              const cplx<T>* __restrict__ tw, int twlog2) {
  using V = cplx<T>;
  const int nb = n / R;
  const int total = ntile * nb;
  const int step_log = twlog2 - (__builtin_ctz(Ns) + lr);   // NT / (Ns R)
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
        for (int r = 1; r < R; ++r) v[q][r] = c_mul(v[q][r], tw[(r * kk) << step_log]);
      }
      dftR<R, V, T>(v[q]);
      V* dst = buf + t * pitch + ((j - kk) << lr) + kk;
#pragma unroll
      for (int r = 0; r < R; ++r) dst[r * Ns] = v[q][r];
    }
  }
  __syncthreads();
}

// LDS capacity of one block, in complex elements (64 KiB).
template <typename T> constexpr int lds_cap() { return 65536 / (int)sizeof(cplx<T>); }

template <typename T>
__device__ __forceinline__ void fft_body(cplx<T>* __restrict__ data, int n, int log2n, long es, long nbatch, long b_in,
                                         long s_in, long s_out, int tile, const cplx<T>* __restrict__ tw, int twlog2,
                                         long blk, char* smem_raw) {
  using V = cplx<T>;
  constexpr int CAP = lds_cap<T>();
  const int pitch = n + (es == 1 ? 0 : 1);   // pad column tiles so their LDS writes do not share a bank
  V* buf = reinterpret_cast<V*>(smem_raw);
  const long b0 = blk * tile;
  const int ntile = (int)min((long)tile, nbatch - b0);
  const int total = tile * n;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int t, e;
    if (es == 1) { t = idx / n; e = idx - t * n; }
    else { e = idx / tile; t = idx - e * tile; }
    if (t < ntile) {
      const long b = b0 + t;
      const long base = (b / b_in) * s_out + (b % b_in) * s_in;
      buf[t * pitch + e] = data[base + (long)e * es];
    }
  }
  __syncthreads();
  // radix-8 passes, then one radix-4 or radix-2 pass for the remaining factor
  int Ns = 1, rem = log2n;
  while (rem >= 3) {
    stockham_pass<T, 8, CAP / (8 * 256)>(buf, n, pitch, ntile, Ns, 3, tw, twlog2);
    Ns <<= 3;
    rem -= 3;
  }
  if (rem == 2) stockham_pass<T, 4, CAP / (4 * 256)>(buf, n, pitch, ntile, Ns, 2, tw, twlog2);
  else if (rem == 1) stockham_pass<T, 2, CAP / (2 * 256)>(buf, n, pitch, ntile, Ns, 1, tw, twlog2);
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    int t, e;
    if (es == 1) { t = idx / n; e = idx - t * n; }
    else { e = idx / tile; t = idx - e * tile; }
    if (t < ntile) {
      const long b = b0 + t;
      const long base = (b / b_in) * s_out + (b % b_in) * s_in;
      data[base + (long)e * es] = buf[t * pitch + e];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fft(cplx<T>* __restrict__ data, int n, int log2n, long es, long nbatch,
                                             long b_in, long s_in, long s_out, int tile,
                                             const cplx<T>* __restrict__ tw, int twlog2) {
  extern __shared__ char smem_raw[];
  fft_body<T>(data, n, log2n, es, nbatch, b_in, s_in, s_out, tile, tw, twlog2, blockIdx.x, smem_raw);
}

// Several independent batched transforms (segments, e.g. one per instance, of
// different lengths) in one launch; block b belongs to the last segment whose
// first block is <= b.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_multi(cplx<T>* __restrict__ base, const FftSeg* __restrict__ segs,
                                                   int nseg, const cplx<T>* __restrict__ tw, int twlog2) {
  extern __shared__ char smem_raw[];
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].blk0 <= (long)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const FftSeg g = segs[lo];
  fft_body<T>(base + g.off, g.n, g.log2n, g.es, g.nbatch, g.b_in, g.s_in, g.s_out, g.tile, tw, twlog2,
              (long)blockIdx.x - g.blk0, smem_raw);
}

template <typename T>
hipError_t fft_impl(Plan& P, void* data, int n, long es, long nbatch, long b_in, long s_in, long s_out) {
  if (n <= 1 || nbatch <= 0) return hipSuccess;
  const int log2n = __builtin_ctz((unsigned)n);
  int tile = fft_tile(P, n, es == 1, nbatch);
  const size_t shm = (size_t)tile * (n + (es == 1 ? 0 : 1)) * sizeof(cplx<T>);
  const long nblk = (nbatch + tile - 1) / tile;
  const cplx<T>* tw = nullptr;
  if constexpr (sizeof(T) == 8) tw = P.tw; else tw = P.twf;
  hipLaunchKernelGGL(k_fft<T>, dim3((unsigned)nblk), dim3(256), shm, P.stream, static_cast<cplx<T>*>(data), n, log2n,
                     es, nbatch, b_in, s_in, s_out, tile, tw, P.twlog2);
  return hipGetLastError();
}

template <typename T>
hipError_t fft_multi_impl(Plan& P, void* base, const FftSeg* dsegs, int nseg, long nblocks, long lds_elems) {
  const size_t shm = (size_t)lds_elems * sizeof(cplx<T>);
  const cplx<T>* tw = nullptr;
  if constexpr (sizeof(T) == 8) tw = P.tw; else tw = P.twf;
  hipLaunchKernelGGL(k_fft_multi<T>, dim3((unsigned)nblocks), dim3(256), shm, P.stream, static_cast<cplx<T>*>(base),
                     dsegs, nseg, tw, P.twlog2);
  return hipGetLastError();
}

}  // namespace

// Transforms per block: as many as fill 64 KiB of LDS (one in-place buffer), at
// most 64, unless the autotuner has recorded a faster choice for this length
// and axis.  Never more than fit: the passes hold at most 64 KiB / (R * 256)
// butterflies per thread in registers.
int fft_tile(const Plan& P, int n, bool rows, long nbatch) {
  const int pitch = n + (rows ? 0 : 1);
  const int cap = (int)(65536 / P.esize) / pitch;
  int tile = 0;
  const int key = (n << 2) | (rows ? 1 : 0) | (P.p.prec == QPGF_C64 ? 2 : 0);
  auto it = P.fft_tiles.find(key);
  if (it != P.fft_tiles.end()) tile = it->second;
  if (tile <= 0 || tile > cap) {
    tile = cap;
    if (tile > 64) tile = 64;
    // columns: whole aligned groups of adjacent columns
    if (!rows) tile = 1 << (31 - __builtin_clz((unsigned)tile));
    // keep at least ~1024 blocks in flight (4 per CU) while groups stay >= 64 bytes
    const int min_tile = rows ? 1 : std::max(1, (int)(64 / P.esize));
    while (tile > min_tile && (nbatch + tile - 1) / tile < 1024) tile >>= 1;
  }
  if (tile < 1) tile = 1;
  if (tile > nbatch) tile = (int)nbatch;
  return tile;
}

hipError_t launch_fft_multi(Plan& P, void* base, const FftSeg* dsegs, int nseg, long nblocks, long lds_elems) {
  return P.p.prec == QPGF_C128 ? fft_multi_impl<double>(P, base, dsegs, nseg, nblocks, lds_elems)
                               : fft_multi_impl<float>(P, base, dsegs, nseg, nblocks, lds_elems);
}

hipError_t launch_fft(Plan& P, void* data, int n, long es, long nbatch, long b_in, long s_in, long s_out) {
  return P.p.prec == QPGF_C128 ? fft_impl<double>(P, data, n, es, nbatch, b_in, s_in, s_out)
                               : fft_impl<float>(P, data, n, es, nbatch, b_in, s_in, s_out);
}

}  // namespace qpgf
