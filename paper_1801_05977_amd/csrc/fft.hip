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

#include "fft_device.h"
#include "qpgf_internal.h"

namespace qpgf {

namespace {

using namespace fftdev;

template <typename T>
__device__ __forceinline__ void fft_body(cplx<T>* __restrict__ data, int n, long es, long nbatch, long b_in,
                                         long s_in, long s_out, int tile, const cplx<T>* __restrict__ tw, int ntw,
                                         long blk, char* smem_raw) {
  using V = cplx<T>;
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
  if (fft_twiddles_in_lds(tile, pitch, n, sizeof(V))) {
    // the n twiddles of this length, read once into LDS after the block's data
    V* twl = buf + tile * pitch;
    const int stride = ntw / n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) twl[j] = tw[(long)j * stride];
    __syncthreads();
    inverse_dft_lds<T>(buf, n, pitch, ntile, twl, n);
  } else {
    inverse_dft_lds<T>(buf, n, pitch, ntile, tw, ntw);
  }
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
__global__ __launch_bounds__(256) void k_fft(cplx<T>* __restrict__ data, int n, long es, long nbatch,
                                             long b_in, long s_in, long s_out, int tile,
                                             const cplx<T>* __restrict__ tw, int ntw) {
  extern __shared__ char smem_raw[];
  fft_body<T>(data, n, es, nbatch, b_in, s_in, s_out, tile, tw, ntw, blockIdx.x, smem_raw);
}

// Several independent batched transforms (segments, e.g. one per instance, of
// different lengths) in one launch; block b belongs to the last segment whose
// first block is <= b.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_multi(cplx<T>* __restrict__ base, const FftSeg* __restrict__ segs,
                                                   int nseg, const cplx<T>* __restrict__ tw, int ntw) {
  extern __shared__ char smem_raw[];
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].blk0 <= (long)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const FftSeg g = segs[lo];
  fft_body<T>(base + g.off, g.n, g.es, g.nbatch, g.b_in, g.s_in, g.s_out, g.tile, tw, ntw,
              (long)blockIdx.x - g.blk0, smem_raw);
}

template <typename T>
hipError_t fft_impl(Plan& P, void* data, int n, long es, long nbatch, long b_in, long s_in, long s_out) {
  if (n <= 1 || nbatch <= 0) return hipSuccess;
  int tile = fft_tile(P, n, es == 1, nbatch);
  const int pitch = n + (es == 1 ? 0 : 1);
  const size_t shm = ((size_t)tile * pitch + (fft_twiddles_in_lds(tile, pitch, n, sizeof(cplx<T>)) ? n : 0)) *
                     sizeof(cplx<T>);
  const long nblk = (nbatch + tile - 1) / tile;
  const cplx<T>* tw = nullptr;
  if constexpr (sizeof(T) == 8) tw = P.tw; else tw = P.twf;
  hipLaunchKernelGGL(k_fft<T>, dim3((unsigned)nblk), dim3(256), shm, P.stream, static_cast<cplx<T>*>(data), n,
                     es, nbatch, b_in, s_in, s_out, tile, tw, P.ntw);
  return hipGetLastError();
}

template <typename T>
hipError_t fft_multi_impl(Plan& P, void* base, const FftSeg* dsegs, int nseg, long nblocks, long lds_elems) {
  const size_t shm = (size_t)lds_elems * sizeof(cplx<T>);
  const cplx<T>* tw = nullptr;
  if constexpr (sizeof(T) == 8) tw = P.tw; else tw = P.twf;
  hipLaunchKernelGGL(k_fft_multi<T>, dim3((unsigned)nblocks), dim3(256), shm, P.stream, static_cast<cplx<T>*>(base),
                     dsegs, nseg, tw, P.ntw);
  return hipGetLastError();
}

}  // namespace

// Transforms per block: about 2048 elements, at most 64 transforms and never
// more than fit 64 KiB of LDS (the passes hold at most 64 KiB / (R * 256)
// butterflies per thread in registers), unless the autotuner has recorded a
// faster choice for this length and axis.
int fft_tile(const Plan& P, int n, bool rows, long nbatch) {
  const int pitch = n + (rows ? 0 : 1);
  const int cap = (int)(65536 / P.esize) / pitch;
  int tile = 0;
  const int key = (n << 2) | (rows ? 1 : 0) | (P.p.prec == QPGF_C64 ? 2 : 0);
  auto it = P.fft_tiles.find(key);
  if (it != P.fft_tiles.end()) tile = it->second;
  if (tile <= 0 || tile > cap) {
    // about 2048 elements per block (16 KiB complex64): several blocks per CU,
    // so one block's LDS passes overlap the others' global loads and stores
    // (the autotuner's choices on gfx950 cluster there)
    // column groups of at least 64 bytes so the loads stay coalesced
    const int min_tile = rows ? 1 : std::max(1, (int)(64 / P.esize));
    tile = std::max(1, std::min(cap, std::max(2048 / n, min_tile)));
    if (tile > 64) tile = 64;
    // columns: whole aligned groups of adjacent columns
    if (!rows) tile = 1 << (31 - __builtin_clz((unsigned)tile));
    // keep at least ~1024 blocks in flight (4 per CU)
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
