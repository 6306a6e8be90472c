// Batched inverse DFTs (unnormalised, e^{+2 pi i jp/n}) along one axis of a
// strided array: the grid synthesis of Algorithms 2.1 / 3.1 / 4.1 (steps 1c-1d),
// L_N(x_p) = sum_j L-hat_j e^{i pi j p / N}, with coefficients and grid points
// both stored mod n.  Lengths 2^a r (r = 1, 3, 5, 7): radix-8/4/2 Stockham
// autosort passes and one radix-r pass, staged in LDS.
//
// Batch b of a launch starts at element (b / b_in) * s_out + (b % b_in) * s_in
// and its elements are elem_stride apart.  A block takes `tile` consecutive
// batches: for rows (elem_stride 1) each batch is one contiguous run, for
// columns (s_in 1) the tile's batches are adjacent, so both load coalesced.
// Every thread issues its loads (and stores) 64 bytes at a time before it
// touches LDS, so a block keeps that many bytes per thread in flight instead of
// one value; consecutive tiles go to the same XCD (blocks are dealt to the eight
// XCDs in turn), so the halves of a 128-byte line that two column tiles share
// meet in one L2.
#include <algorithm>

#include "fft_device.h"
#include "qpgf_internal.h"

namespace qpgf {

namespace {

using namespace fftdev;

// global transfers per thread in flight: 64 bytes (8 complex64 or 4 complex128 values, which
// stay in registers; larger arrays of complex128 are placed in scratch memory by the compiler)
template <typename T> constexpr int ld_unroll() { return 64 / (int)sizeof(cplx<T>); }

// Logical block of hardware block b of nblk: the hardware deals blocks to the 8 XCDs in turn,
// so block b runs on XCD b % 8; logical blocks [x per, (x + 1) per) all run on XCD x.
__device__ __forceinline__ long xcd_block(long b, long nblk) {
  const long per = nblk >> 3;
  return b < (per << 3) ? (b & 7) * per + (b >> 3) : b;
}

template <typename T>
__device__ __forceinline__ void fft_body(cplx<T>* __restrict__ data, int n, long es, long nbatch, long b_in,
                                         long s_in, long s_out, int tile, const cplx<T>* __restrict__ tw, int ntw,
                                         long blk, char* smem_raw) {
  using V = cplx<T>;
  constexpr int kLdU = ld_unroll<T>();
  const bool rows = es == 1;
  const int pitch = n + (rows ? 0 : 1);   // pad column tiles so their LDS writes do not share a bank
  V* buf = reinterpret_cast<V*>(smem_raw);
  const long b0 = blk * tile;
  const int ntile = (int)min((long)tile, nbatch - b0);
  const int total = tile * n;
  // element idx of the block's tile: transform t, element e (rows: e fastest; columns: t fastest);
  // 32-bit quotients (the host keeps batches below 2^31)
  // (the global offset, and the LDS offset or -1 beyond the block's transforms, where the global
  // offset is the block's own first element: a lane past the end reloads it, and no other block
  // writes it)
  const unsigned un = (unsigned)n, ut = (unsigned)tile, ubin = (unsigned)b_in;
  struct Loc {
    long g;
    int l;
  };
  const long g0 = (b0 / b_in) * s_out + (b0 % b_in) * s_in;
  auto locate = [&](int idx) -> Loc {
    unsigned t, e;
    if (rows) {
      t = (unsigned)idx / un;
      e = (unsigned)idx - t * un;
    } else {
      e = (unsigned)idx / ut;
      t = (unsigned)idx - e * ut;
    }
    if (idx >= total || (int)t >= ntile) return Loc{g0, -1};
    const unsigned b = (unsigned)b0 + t, q = b / ubin;
    return Loc{(long)q * s_out + (long)(b - q * ubin) * s_in + (long)e * es, (int)(t * (unsigned)pitch + e)};
  };
  // (every lane loads, so no load sits in a branch whose join would wait for it)
  for (int i0 = 0; i0 < total; i0 += kLdU * 256) {
    V v[kLdU];
    int o[kLdU];
#pragma unroll
    for (int u = 0; u < kLdU; ++u) {
      const Loc L = locate(i0 + u * 256 + (int)threadIdx.x);
      o[u] = L.l;
      v[u] = data[L.g];
    }
#pragma unroll
    for (int u = 0; u < kLdU; ++u)
      if (o[u] >= 0) buf[o[u]] = v[u];
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
  for (int i0 = 0; i0 < total; i0 += kLdU * 256) {
    V v[kLdU];
    Loc L[kLdU];
#pragma unroll
    for (int u = 0; u < kLdU; ++u) {
      L[u] = locate(i0 + u * 256 + (int)threadIdx.x);
      v[u] = buf[L[u].l >= 0 ? L[u].l : 0];
    }
#pragma unroll
    for (int u = 0; u < kLdU; ++u)
      if (L[u].l >= 0) data[L[u].g] = v[u];
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fft(cplx<T>* __restrict__ data, int n, long es, long nbatch,
                                             long b_in, long s_in, long s_out, int tile,
                                             const cplx<T>* __restrict__ tw, int ntw) {
  extern __shared__ char smem_raw[];
  fft_body<T>(data, n, es, nbatch, b_in, s_in, s_out, tile, tw, ntw, xcd_block(blockIdx.x, gridDim.x), smem_raw);
}

// Several independent batched transforms (segments, e.g. one per instance, of
// different lengths) in one launch; block b belongs to the last segment whose
// first block is <= b.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_multi(cplx<T>* __restrict__ base, const FftSeg* __restrict__ segs,
                                                   int nseg, const cplx<T>* __restrict__ tw, int ntw) {
  extern __shared__ char smem_raw[];
  const long blk = xcd_block(blockIdx.x, gridDim.x);
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].blk0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  const FftSeg g = segs[lo];
  fft_body<T>(base + g.off, g.n, g.es, g.nbatch, g.b_in, g.s_in, g.s_out, g.tile, tw, ntw, blk - g.blk0, smem_raw);
}

// x1 rows of the 3D G_d far slab [s][i2][i1] after its x2 pass.  Row b = s M2 + i2 is zero in every
// column j1 whose terms all fell past the cut at z_s = z0 + s hf (far_band_empty): the x2 pass
// leaves those columns unwritten and here they are taken as zero without being read (their lanes
// load the block's first element, so every lane still loads and no load waits at a branch join).
template <typename T>
__global__ __launch_bounds__(256) void k_fft_far_rows(cplx<T>* __restrict__ data, int n, long nrows, int M2, int tile,
                                                      double k, double a1, double z0, double hf,
                                                      const cplx<T>* __restrict__ tw, int ntw) {
  extern __shared__ char smem_raw[];
  using V = cplx<T>;
  constexpr int kLdU = ld_unroll<T>();
  V* buf = reinterpret_cast<V*>(smem_raw);
  const long b0 = xcd_block(blockIdx.x, gridDim.x) * tile;
  const int ntile = (int)min((long)tile, nrows - b0);
  const int total = tile * n;
  const unsigned un = (unsigned)n, um2 = (unsigned)M2;
  const long g0 = b0 * n;
  V zero;
  zero.x = (T)0;
  zero.y = (T)0;
  for (int i0 = 0; i0 < total; i0 += kLdU * 256) {
    V v[kLdU];
    int o[kLdU];   // LDS offset of a value read; -2 - offset for a zero; -1 past the block's rows
#pragma unroll
    for (int u = 0; u < kLdU; ++u) {
      const int idx = i0 + u * 256 + (int)threadIdx.x;
      const unsigned t = (unsigned)idx / un, e = (unsigned)idx - t * un;
      const bool in = idx < total && (int)t < ntile;
      const unsigned b = (unsigned)b0 + t, s = b / um2;
      const double xi = a1 + (double)((int)e < (n >> 1) ? (int)e : (int)e - n);
      const bool keep = in && !far_band_empty(xi, k, z0, hf, (long)s);
      o[u] = keep ? idx : in ? -2 - idx : -1;
      v[u] = data[keep ? b0 * n + idx : g0];
    }
#pragma unroll
    for (int u = 0; u < kLdU; ++u) {
      if (o[u] >= 0) buf[o[u]] = v[u];
      else if (o[u] <= -2) buf[-2 - o[u]] = zero;
    }
  }
  __syncthreads();
  if (fft_twiddles_in_lds(tile, n, n, sizeof(V))) {
    V* twl = buf + tile * n;
    const int stride = ntw / n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) twl[j] = tw[(long)j * stride];
    __syncthreads();
    inverse_dft_lds<T>(buf, n, n, ntile, twl, n);
  } else {
    inverse_dft_lds<T>(buf, n, n, ntile, tw, ntw);
  }
  for (int i0 = 0; i0 < total; i0 += kLdU * 256) {
    V v[kLdU];
    int o[kLdU];
#pragma unroll
    for (int u = 0; u < kLdU; ++u) {
      const int idx = i0 + u * 256 + (int)threadIdx.x;
      o[u] = idx < ntile * n ? idx : -1;
      v[u] = buf[o[u] >= 0 ? o[u] : 0];
    }
#pragma unroll
    for (int u = 0; u < kLdU; ++u)
      if (o[u] >= 0) data[g0 + o[u]] = v[u];
  }
}

// x2 columns of the Maxwell far slab [f][s][i2][i1] after its x1 pass, `tile` adjacent columns per
// block.  Column (f, s, i1) is zero at every j2 whose terms all fell past the cut at z_s = z0 + s hf
// (far_band_empty): the x1 pass leaves those rows unwritten and here they are taken as zero without
// being read, as in k_fft_far_rows.  Batch b: plane q = b / M1 (field q / S, slice q % S), column b % M1.
template <typename T>
__global__ __launch_bounds__(256) void k_fft_far_cols(cplx<T>* __restrict__ data, int n, int M1, int S, long nbatch,
                                                      int tile, double k, double a2, double z0, double hf,
                                                      const cplx<T>* __restrict__ tw, int ntw) {
  extern __shared__ char smem_raw[];
  using V = cplx<T>;
  constexpr int kLdU = ld_unroll<T>();
  const int pitch = n + 1;
  V* buf = reinterpret_cast<V*>(smem_raw);
  const long b0 = xcd_block(blockIdx.x, gridDim.x) * tile;
  const int ntile = (int)min((long)tile, nbatch - b0);
  const int total = tile * n;
  const unsigned ut = (unsigned)tile, um1 = (unsigned)M1, us = (unsigned)S;
  const long plane = (long)M1 * n;
  const long g0 = (b0 / M1) * plane + (b0 % M1);
  auto gofs = [&](unsigned t, unsigned e) -> long {
    const unsigned b = (unsigned)b0 + t, q = b / um1;
    return (long)q * plane + (long)e * M1 + (b - q * um1);
  };
  V zero;
  zero.x = (T)0;
  zero.y = (T)0;
  for (int i0 = 0; i0 < total; i0 += kLdU * 256) {
    V v[kLdU];
    int o[kLdU];   // LDS offset of a value read; -2 - offset for a zero; -1 past the block's columns
#pragma unroll
    for (int u = 0; u < kLdU; ++u) {
      const int idx = i0 + u * 256 + (int)threadIdx.x;
      const unsigned e = (unsigned)idx / ut, t = (unsigned)idx - e * ut;
      const bool in = idx < total && (int)t < ntile;
      const unsigned s = (((unsigned)b0 + t) / um1) % us;
      const double xi = a2 + (double)((int)e < (n >> 1) ? (int)e : (int)e - n);
      const bool keep = in && !far_band_empty(xi, k, z0, hf, (long)s);
      const int l = (int)(t * (unsigned)pitch + e);
      o[u] = keep ? l : in ? -2 - l : -1;
      v[u] = data[keep ? gofs(t, e) : g0];
    }
#pragma unroll
    for (int u = 0; u < kLdU; ++u) {
      if (o[u] >= 0) buf[o[u]] = v[u];
      else if (o[u] <= -2) buf[-2 - o[u]] = zero;
    }
  }
  __syncthreads();
  if (fft_twiddles_in_lds(tile, pitch, n, sizeof(V))) {
    V* twl = buf + tile * pitch;
    const int stride = ntw / n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) twl[j] = tw[(long)j * stride];
    __syncthreads();
    inverse_dft_lds<T>(buf, n, pitch, ntile, twl, n);
  } else {
    inverse_dft_lds<T>(buf, n, pitch, ntile, tw, ntw);
  }
  for (int i0 = 0; i0 < total; i0 += kLdU * 256) {
    V v[kLdU];
    long g[kLdU];
    int o[kLdU];
#pragma unroll
    for (int u = 0; u < kLdU; ++u) {
      const int idx = i0 + u * 256 + (int)threadIdx.x;
      const unsigned e = (unsigned)idx / ut, t = (unsigned)idx - e * ut;
      const bool in = idx < total && (int)t < ntile;
      o[u] = in ? (int)(t * (unsigned)pitch + e) : -1;
      g[u] = in ? gofs(t, e) : g0;
      v[u] = buf[o[u] >= 0 ? o[u] : 0];
    }
#pragma unroll
    for (int u = 0; u < kLdU; ++u)
      if (o[u] >= 0) data[g[u]] = v[u];
  }
}

template <typename T>
hipError_t fft_impl(Plan& P, void* data, int n, long es, long nbatch, long b_in, long s_in, long s_out) {
  if (n <= 1 || nbatch <= 0) return hipSuccess;
  if (nbatch + 64 >= (1L << 31)) return hipErrorInvalidValue;   // 32-bit batch indices in the kernel
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

// Transforms per block: about 32 KiB of data, at most 64 transforms and never
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
    // about 32 KiB per block (4096 complex64 or 2048 complex128 elements): several blocks per
    // CU, so one block's LDS passes overlap the others' global loads and stores (measured on
    // gfx950: length-512 rows of complex64 move 3.5 TB/s at 8 per block, 2.8 TB/s at 4)
    // column groups of at least 64 bytes so the loads stay coalesced
    const int min_tile = rows ? 1 : std::max(1, (int)(64 / P.esize));
    tile = std::max(1, std::min(cap, std::max((int)(32768 / P.esize) / n, min_tile)));
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

hipError_t launch_fft_far_rows(Plan& P, double k, double a1) {
  const int n = P.Mf1;
  const long nrows = (long)P.Mf2 * P.S;
  if (n <= 1 || nrows <= 0) return hipSuccess;
  if (nrows + 64 >= (1L << 31)) return hipErrorInvalidValue;   // 32-bit row indices in the kernel
  const int tile = fft_tile(P, n, true, nrows);
  const long nblk = (nrows + tile - 1) / tile;
  if (P.p.prec == QPGF_C128) {
    const size_t shm = ((size_t)tile * n + (fft_twiddles_in_lds(tile, n, n, sizeof(double2)) ? n : 0)) * sizeof(double2);
    hipLaunchKernelGGL(k_fft_far_rows<double>, dim3((unsigned)nblk), dim3(256), shm, P.stream,
                       static_cast<double2*>(P.far), n, nrows, P.Mf2, tile, k, a1, P.fz0, P.hf, P.tw, P.ntw);
  } else {
    const size_t shm = ((size_t)tile * n + (fft_twiddles_in_lds(tile, n, n, sizeof(float2)) ? n : 0)) * sizeof(float2);
    hipLaunchKernelGGL(k_fft_far_rows<float>, dim3((unsigned)nblk), dim3(256), shm, P.stream,
                       static_cast<float2*>(P.far), n, nrows, P.Mf2, tile, k, a1, P.fz0, P.hf, P.twf, P.ntw);
  }
  return hipGetLastError();
}

hipError_t launch_fft_far_cols(Plan& P, double k, double a2) {
  const int n = P.Mf2;
  const long nbatch = (long)P.Mf1 * P.S * P.nfo;
  if (n <= 1 || nbatch <= 0) return hipSuccess;
  if (nbatch + 64 >= (1L << 31)) return hipErrorInvalidValue;   // 32-bit batch indices in the kernel
  const int tile = fft_tile(P, n, false, nbatch), pitch = n + 1;
  const long nblk = (nbatch + tile - 1) / tile;
  if (P.p.prec == QPGF_C128) {
    const size_t shm =
        ((size_t)tile * pitch + (fft_twiddles_in_lds(tile, pitch, n, sizeof(double2)) ? n : 0)) * sizeof(double2);
    hipLaunchKernelGGL(k_fft_far_cols<double>, dim3((unsigned)nblk), dim3(256), shm, P.stream,
                       static_cast<double2*>(P.far), n, P.Mf1, P.S, nbatch, tile, k, a2, P.fz0, P.hf, P.tw, P.ntw);
  } else {
    const size_t shm =
        ((size_t)tile * pitch + (fft_twiddles_in_lds(tile, pitch, n, sizeof(float2)) ? n : 0)) * sizeof(float2);
    hipLaunchKernelGGL(k_fft_far_cols<float>, dim3((unsigned)nblk), dim3(256), shm, P.stream,
                       static_cast<float2*>(P.far), n, P.Mf1, P.S, nbatch, tile, k, a2, P.fz0, P.hf, P.twf, P.ntw);
  }
  return hipGetLastError();
}

}  // namespace qpgf
