// Calculation step of Algorithms 2.1 / 3.1 / 4.1 for many targets: reduce each
// target to the period cell (step 2c), branch on |x_t| <= c (step 2b),
// interpolate the near grid with the tensor-product 4-point Lagrange rule
// (16 / 64 nodes, step 2d), add back the removed singular part in FP64 and apply
// the quasi-periodic phase (steps 2e-2f; Algorithm 4.1 steps 2e-2i).  Far targets
// take the eigenfunction series (step 2b), summed on the far slab and interpolated
// there with the 8-point rule per axis (64 / 512 nodes).
#include <algorithm>
#include <cstring>

#include "qpgf_internal.h"

namespace qpgf {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

struct GArgs {
  double k, a1, a2, c, c_tilde, eps, rmin;
  double k2;               // second wavenumber (differences of second derivatives, 2D)
  int M1, M2, M3;          // 2D: M2 = transverse size, M3 = 1
  double h1, h2, h3;       // 2D: h2 = transverse spacing
  double ih1, ih2, ih3;    // reciprocals of the spacings
  double hf, ihf;          // far-slab slice spacing and its reciprocal
  double fz0;              // far-slab first slice, c - (fp/2 - 1) hf
  int S;                   // far-slab slices
  int fp;                  // far-slab interpolation points per axis (4 or 8)
  int Mf1, Mf2;            // far-slab periodic sizes (Mf2 = 1 in 2D)
  double ihf1, ihf2;       // reciprocals of the far slab's periodic spacings 2 pi / Mf
  long fs, ffs;            // field strides (near, far)
  int smooth;              // 1: return the interpolated smooth part L_N only (near branch)
  int sing_order;          // 2D G: degree of the removed Taylor factor of the log singularity (1..3)
  int quad;                // 2D G, complex64: the near grid is node quads (4 x1-neighbours per node)
  int far_layout;          // 2D far slab: 0 fields apart [f][s][i1], 1 node quads, 2 fields interleaved
  // 2D kinds, ring_interp: bit i of ring_mask marks target i (a near target with
  // ring_lo < r < ring_hi) for the ring pass
  unsigned long long* ring_mask;
  double ring_lo, ring_hi;
};

// cubic Lagrange weights at nodes -1, 0, 1, 2 (W = float on the complex64
// path: the fraction is formed in FP64, the weights in FP32)
template <typename W>
__device__ __forceinline__ void lag4(W f, W w[4]) {
  const W fm1 = f - W(1), fm2 = f - W(2), fp1 = f + W(1);
  w[0] = -f * fm1 * fm2 * W(1.0 / 6.0);
  w[1] = fp1 * fm1 * fm2 * W(0.5);
  w[2] = -fp1 * f * fm2 * W(0.5);
  w[3] = fp1 * f * fm1 * W(1.0 / 6.0);
}

// x = 2 pi n + t, t in [-pi, pi) (up to rounding at the cell edge, where the
// grid is periodic and the singular part vanishes, so either cell gives G)
__device__ __forceinline__ double reduce_cell(double x, double& n) {
  n = floor((x + kPi) * (0.5 / kPi));
  return x - 2.0 * kPi * n;
}

template <typename T> struct Acc;
template <> struct Acc<double> {
  double2 v;
  __device__ Acc() : v(make_double2(0.0, 0.0)) {}
  __device__ void add(double w, double2 g) { v.x = fma(w, g.x, v.x); v.y = fma(w, g.y, v.y); }
  __device__ double2 get() const { return v; }
};
template <> struct Acc<float> {
  float2 v;
  __device__ Acc() : v(make_float2(0.f, 0.f)) {}
  __device__ void add(float w, float2 g) { v.x = fmaf(w, g.x, v.x); v.y = fmaf(w, g.y, v.y); }
  __device__ double2 get() const { return make_double2(v.x, v.y); }
};

template <typename T> __device__ __forceinline__ void store_out(cplx<T>* p, long i, double2 v);
template <> __device__ __forceinline__ void store_out<double>(double2* p, long i, double2 v) { p[i] = v; }
template <> __device__ __forceinline__ void store_out<float>(float2* p, long i, double2 v) {
  p[i] = make_float2((float)v.x, (float)v.y);
}

__device__ __forceinline__ double2 nan2() { return mk(__builtin_nan(""), __builtin_nan("")); }

// P-point Lagrange weights at nodes -(P/2 - 1) .. P/2 for the fraction f in [0, 1) (the far
// branch): w_m = prod_{n != m} (f - node_n) / prod_{n != m} (node_m - node_n), products before and
// after m; prod_{n != m} (m - n) = (-1)^(P-1-m) m! (P-1-m)!.
template <int P>
__host__ __device__ constexpr double lag_inv_den(int m) {
  double d = 1.0;
  for (int n = 0; n < P; ++n)
    if (n != m) d *= (double)(m - n);
  return 1.0 / d;
}
// (node m at offset m - LOW from the base node; LOW = P/2 - 1 centres an even rule on the
// target's cell)
template <typename W, int P, int LOW = P / 2 - 1>
__device__ __forceinline__ void lagp(W f, W w[P]) {
  W g[P], pre[P], suf[P];
#pragma unroll
  for (int m = 0; m < P; ++m) g[m] = f + W(LOW - m);
  pre[0] = W(1);
#pragma unroll
  for (int m = 1; m < P; ++m) pre[m] = pre[m - 1] * g[m - 1];
  suf[P - 1] = W(1);
#pragma unroll
  for (int m = P - 2; m >= 0; --m) suf[m] = suf[m + 1] * g[m + 1];
#pragma unroll
  for (int m = 0; m < P; ++m) w[m] = pre[m] * suf[m] * W(lag_inv_den<P>(m));
}

// Far-slab slice stencil of |x_t| = z: base slice s0 = floor((z - fz0) / hf) (>= fp/2 - 1 for
// z > c) and the fraction; false when the fp slices s0 - (fp/2 - 1) .. s0 + fp/2 leave the slab.
__device__ __forceinline__ bool far_slice(const GArgs& A, double z, double& s0, double& f) {
  const double v = (z - A.fz0) * A.ihf;
  s0 = floor(v);
  if (!(s0 <= A.S - 1 - A.fp / 2)) return false;
  s0 = fmax(s0, (double)(A.fp / 2 - 1));
  f = v - s0;
  return true;
}

// Number of results per target: G_d, or the six Maxwell entries.
template <int NF> struct NOut { static constexpr int v = NF == 1 ? 1 : 6; };

// ---------------------------------------------------------------------------
// 3D near branch (Algorithm 3.1 / 4.1 steps 2c-2i)
// ---------------------------------------------------------------------------
// The stencil of one near target: cell reduction (step 2c), base nodes and the three
// 4-point weight sets (the tricubic rule of step 2d).
template <typename T>
struct Near3 {
  double t1, t2, n1, n2;
  int p1, p2, p3;
  T w1[4], w2[4], w3[4];
};

template <typename T>
__device__ __forceinline__ void near3_stencil(const GArgs& A, double x1, double x2, double x3, Near3<T>& s) {
  s.t1 = reduce_cell(x1, s.n1);
  s.t2 = reduce_cell(x2, s.n2);
  const double u1 = s.t1 * A.ih1, q1 = floor(u1);
  const double u2 = s.t2 * A.ih2, q2 = floor(u2);
  const double u3 = x3 * A.ih3, q3 = floor(u3);
  lag4<T>((T)(u1 - q1), s.w1);
  lag4<T>((T)(u2 - q2), s.w2);
  lag4<T>((T)(u3 - q3), s.w3);
  s.p1 = (int)q1;
  s.p2 = (int)q2;
  s.p3 = (int)q3;
}

// 64-point stencil sums of the NF near fields from global memory (periodic in every axis).
template <typename T, int NF>
__device__ __forceinline__ void near3_sum_global(const GArgs& A, const cplx<T>* __restrict__ grid, const Near3<T>& s,
                                                 double2 L[NF]) {
  Acc<T> acc[NF];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const long i3 = (long)((s.p3 - 1 + c) & (A.M3 - 1));
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long row = (i3 * A.M2 + ((s.p2 - 1 + b) & (A.M2 - 1))) * (long)A.M1;
      const T wcb = s.w3[c] * s.w2[b];
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const T w = wcb * s.w1[a];
        const long o = row + ((s.p1 - 1 + a) & (A.M1 - 1));
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f].add(w, grid[f * A.fs + o]);
      }
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) L[f] = acc[f].get();
}

// From the stencil sums L of the NF near fields to the result: phase e^{i alpha.x'} (step 2f,
// with the original coordinates), exact FP64 add-back of the removed singular part
// psi = e^{ikr} Y(r) / (4 pi r) and of its Hessian (steps 2e, 2g-2h), and the Maxwell tensor
// GG_pq = delta_pq G_d + k^-2 d_p d_q G_d (eq. 4.1, step 2i).  NF = kMxF: fields 11 22 33 12 13 23;
// NF = kMxT: 11 22 12 13 23 with GG_33 = 2 G_d - GG_11 - GG_22.
template <typename T, int NF>
__device__ __forceinline__ void near3_finish(const GArgs& A, double x1, double x2, double x3, const Near3<T>& s,
                                             const double2 L[NF], double2* res, uint8_t& fl) {
  constexpr int NO = NOut<NF>::v;
  if (A.smooth) {
    // the smooth part L_N(t) of Algorithm 3.1 step 2d
#pragma unroll
    for (int o = 0; o < NO; ++o) res[o] = L[o < NF ? o : 0];
    return;
  }
  double ps, pc;
  sincos(A.a1 * x1 + A.a2 * x2, &ps, &pc);
  const double2 phase = mk(pc, ps);
  double2 G[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) G[f] = cmul(phase, L[f]);
  const double r2 = s.t1 * s.t1 + s.t2 * s.t2 + x3 * x3;
  if (r2 <= A.rmin * A.rmin || r2 == 0.0) {
    fl |= 1;
#pragma unroll
    for (int o = 0; o < NO; ++o) res[o] = nan2();
    return;
  }
  if (r2 < 4.0 * A.eps * A.eps) {
    // the square root only inside the support of the singular part
    const double r = sqrt(r2);
    double sn, cn;
    sincos(A.k * r, &sn, &cn);
    const double2 g = cscale(mk(cn, sn), 1.0 / (4.0 * kPi * r));
    double ls, lc;
    sincospi(2.0 * (A.a1 * s.n1 + A.a2 * s.n2), &ls, &lc);
    const double2 lat = mk(lc, ls);
    const double Y = cut_Y(r, A.eps);
    G[0] = cadd(G[0], cmul(lat, cscale(g, Y)));
    if (NF > 1) {
      // psi', psi'' (radial); d_p d_q psi = psi'' t_p t_q / r^2 + psi' (delta_pq / r - t_p t_q / r^3)
      const double Y1 = cut_Y1(r, A.eps), Y2 = cut_Y2(r, A.eps);
      const double2 ikr = mk(-1.0 / r, A.k);  // ik - 1/r
      const double2 g1 = cmul(g, ikr);
      const double2 g2 = cmul(g, cadd(cmul(ikr, ikr), mk(1.0 / (r * r), 0.0)));
      const double2 d1 = cadd(cscale(g1, Y), cscale(g, Y1));
      const double2 d2 = cadd(cadd(cscale(g2, Y), cscale(g1, 2.0 * Y1)), cscale(g, Y2));
      const double t[3] = {s.t1, s.t2, x3};
      const int P[6] = {0, 1, 2, 0, 0, 1}, Qp[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
      for (int e = 0, f = 1; e < 6; ++e) {
        if (NF == kMxT && e == 2) continue;
        const double tp = t[P[e]], tq = t[Qp[e]];
        const double a = tp * tq / r2;
        const double bc = ((P[e] == Qp[e]) ? 1.0 / r : 0.0) - tp * tq / (r2 * r);
        G[f] = cadd(G[f], cmul(lat, cadd(cscale(d2, a), cscale(d1, bc))));
        ++f;
      }
    }
  }
  if (NF == 1) {
    res[0] = G[0];
  } else {
    const double ik2 = 1.0 / (A.k * A.k);
    res[0] = cadd(G[0], cscale(G[1], ik2));
    res[1] = cadd(G[0], cscale(G[2], ik2));
    if (NF == kMxF) {
      res[2] = cadd(G[0], cscale(G[3], ik2));
#pragma unroll
      for (int o = 3; o < 6; ++o) res[o] = cscale(G[o + 1], ik2);
    } else {
      // the trace variant: tr GG = 3 G_d + k^-2 Laplacian G_d = 2 G_d (the Helmholtz equation)
      res[2] = csub(cscale(G[0], 2.0), cadd(res[0], res[1]));
#pragma unroll
      for (int o = 3; o < 6; ++o) res[o] = cscale(G[o], ik2);
    }
  }
}

// ---------------------------------------------------------------------------
// 3D far branch (step 2b: the series (1.3), and for Maxwell its term-wise derivatives)
// ---------------------------------------------------------------------------
// The far slab holds the series on its own periodic grid (Mf1 x Mf2, spacings 2 pi / Mf)
// at slices z_s = fz0 + s hf: G_d, or the six tensor entries GG_pq (13 and 23 for x3 > 0).
// FP = far_points<T>() interpolation points per axis.
template <typename T, int FP = far_points<T>(), int FPT = FP>
struct Far3 {
  int p1, p2, s0;
  T w1[FP], w2[FPT], w3[FPT];
};

// false: |x3| beyond the slab.  FPT points along x2 and x3 (FPT = FP - 1: the first FPT nodes of
// the FP-point rows, nodes -(FP/2 - 1) .. FPT - FP/2)
template <typename T, int FP = far_points<T>(), int FPT = FP>
__device__ __forceinline__ bool far3_stencil(const GArgs& A, double x1, double x2, double x3, Far3<T, FP, FPT>& s) {
  double s0, f3;
  if (!far_slice(A, fabs(x3), s0, f3)) return false;
  double n;
  const double u1 = reduce_cell(x1, n) * A.ihf1, q1 = floor(u1);
  const double u2 = reduce_cell(x2, n) * A.ihf2, q2 = floor(u2);
  lagp<T, FP>((T)(u1 - q1), s.w1);
  lagp<T, FPT, FP / 2 - 1>((T)(u2 - q2), s.w2);
  lagp<T, FPT, FP / 2 - 1>((T)f3, s.w3);
  s.p1 = (int)q1;
  s.p2 = (int)q2;
  s.s0 = (int)s0;
  return true;
}

// FP^3-point stencil sums of the NFO far fields from global memory.
template <typename T, int NFO, int FP = far_points<T>()>
__device__ __forceinline__ void far3_sum_global(const GArgs& A, const cplx<T>* __restrict__ far,
                                                const Far3<T, FP>& s, double2 L[NFO]) {
  constexpr int LO = FP / 2 - 1;
  Acc<T> acc[NFO];
  // the slice loop stays rolled; its weight is the head of a copy shifted each step (static
  // indices only, so the weights stay in registers)
  T w3[FP];
#pragma unroll
  for (int m = 0; m < FP; ++m) w3[m] = s.w3[m];
#pragma unroll 1
  for (int c = 0; c < FP; ++c) {
    const T wc = w3[0];
#pragma unroll
    for (int m = 0; m < FP - 1; ++m) w3[m] = w3[m + 1];
    const long i3 = s.s0 - LO + c;
#pragma unroll
    for (int b = 0; b < FP; ++b) {
      const long row = (i3 * A.Mf2 + ((s.p2 - LO + b) & (A.Mf2 - 1))) * (long)A.Mf1;
      const T wcb = wc * s.w2[b];
#pragma unroll
      for (int a = 0; a < FP; ++a) {
        const T w = wcb * s.w1[a];
        const long o = row + ((s.p1 - LO + a) & (A.Mf1 - 1));
#pragma unroll
        for (int f = 0; f < NFO; ++f) acc[f].add(w, far[f * A.ffs + o]);
      }
    }
  }
#pragma unroll
  for (int f = 0; f < NFO; ++f) L[f] = acc[f].get();
}

// From the far sums to the result: the phase e^{i alpha.x'}, and sgn(x3) for GG_13, GG_23
// (d/dx3 of e^{i beta |x3|}).
template <int NFO>
__device__ __forceinline__ void far3_finish(const GArgs& A, double x1, double x2, double x3, const double2 L[NFO],
                                            double2* res) {
  double ps, pc;
  sincos(A.a1 * x1 + A.a2 * x2, &ps, &pc);
  const double2 phase = mk(pc, ps);
#pragma unroll
  for (int o = 0; o < NFO; ++o) res[o] = cmul(phase, L[o]);
  if (NFO == kMxO && x3 < 0.0) {
    res[4] = cscale(res[4], -1.0);
    res[5] = cscale(res[5], -1.0);
  }
}

// One target from global memory, either branch (unsorted targets, the tiled kernels'
// overflow and the key of non-finite or out-of-slab targets).  NFO = far fields.
template <typename T, int NF>
__device__ __forceinline__ void eval3d_global(const GArgs& A, const cplx<T>* __restrict__ grid,
                                              const cplx<T>* __restrict__ far, double x1, double x2, double x3,
                                              double2* res, uint8_t& fl) {
  constexpr int NO = NOut<NF>::v;
  fl = 0;
  if (!(isfinite(x1) && isfinite(x2) && isfinite(x3))) {
    fl = 8;
#pragma unroll
    for (int o = 0; o < NO; ++o) res[o] = nan2();
    return;
  }
  if (fabs(x3) <= A.c) {
    Near3<T> s;
    near3_stencil<T>(A, x1, x2, x3, s);
    double2 L[NF];
    near3_sum_global<T, NF>(A, grid, s, L);
    near3_finish<T, NF>(A, x1, x2, x3, s, L, res, fl);
    return;
  }
  fl |= 2;
  Far3<T> s;
  if (A.smooth || !far3_stencil<T>(A, x1, x2, x3, s)) {
    if (!A.smooth) fl |= 4;
#pragma unroll
    for (int o = 0; o < NO; ++o) res[o] = nan2();
    return;
  }
  double2 L[NO];
  far3_sum_global<T, NO>(A, far, s, L);
  far3_finish<NO>(A, x1, x2, x3, L, res);
}

// 3D, unsorted targets: one thread per target, stencils read from global memory.
template <typename T, int NF>
__global__ __launch_bounds__(256) void k_gather3d(GArgs A, const cplx<T>* __restrict__ grid,
                                                  const cplx<T>* __restrict__ far, const double* __restrict__ x,
                                                  long T_, cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T_) return;
  constexpr int NO = NOut<NF>::v;
  double2 res[NO];
  uint8_t fl;
  eval3d_global<T, NF>(A, grid, far, x[3 * i], x[3 * i + 1], x[3 * i + 2], res, fl);
#pragma unroll
  for (int o = 0; o < NO; ++o) store_out<T>(out, i * NO + o, res[o]);
  if (flags) flags[i] = fl;
}

// ---------------------------------------------------------------------------
// Tiled gathers over targets sorted by grid tile.  Keys (tile_key): near tiles
// (b3 nt2 + b2) nt1 + b1 in [0, nnear); far tiles nnear + (b3 fnt2 + b2) fnt1 + b1;
// the last key holds non-finite and out-of-slab targets.  A near tile covers 2^tb
// nodes per axis and its targets' 4-point stencils lie in the (2^tb + 3)^3 footprint
// starting one node before it; a far tile's 8-point stencils lie in (2^ftb + 7)^3
// starting three nodes before it.
// ---------------------------------------------------------------------------
// A target in tile order: coordinates and caller index in one aligned 32-byte record.
struct alignas(32) TRec {
  double x, y, z;
  uint32_t i, pad;
};

struct TileArgs {
  int tb1, tb2, tb3;       // near tile edge = 1 << tb
  int nt1, nt2, nt3n;      // near tiles along x1, x2, x3
  int ftb1, ftb2, ftb3;    // far tile edge
  int fnt1, fnt2, fnt3;    // far tiles along x1, x2 and the slab's slices
  int nnear, nfar, nkeys;  // nkeys = nnear + nfar + 1
};

// 64-point stencil sum of one field from an LDS footprint with row length F1
// and F2 rows per slice; base points at node (p1 - 1, p2 - 1, p3 - 1).
template <typename T, int F1, int F2>
__device__ __forceinline__ double2 lds_sum(const cplx<T>* base, const T a1[4], const T a2[4], const T a3[4]) {
  T accx = 0, accy = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    T px = 0, py = 0;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const cplx<T>* row = base + (c * F2 + b) * F1;
      T rx = 0, ry = 0;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const cplx<T> v = row[a];
        rx += a1[a] * v.x;
        ry += a1[a] * v.y;
      }
      px += a2[b] * rx;
      py += a2[b] * ry;
    }
    accx += a3[c] * px;
    accy += a3[c] * py;
  }
  return mk((double)accx, (double)accy);
}

// FP^3-point stencil sum of one far field from an LDS footprint (rows of F1, F2 rows per slice).
template <typename T, int F1, int F2, int FP>
__device__ __forceinline__ double2 lds_sump(const cplx<T>* base, const T a1[FP], const T a2[FP], const T a3[FP]) {
  T accx = 0, accy = 0;
  // slices in a rolled loop (the slice weight shifted into place, as in far3_sum_global); rows and
  // nodes unrolled, so every LDS address is the slice base plus an immediate offset
  T w3[FP];
#pragma unroll
  for (int m = 0; m < FP; ++m) w3[m] = a3[m];
#pragma unroll 1
  for (int c = 0; c < FP; ++c) {
    const T wc = w3[0];
#pragma unroll
    for (int m = 0; m < FP - 1; ++m) w3[m] = w3[m + 1];
    const cplx<T>* slice = base + c * (F2 * F1);
    T px = 0, py = 0;
#pragma unroll
    for (int b = 0; b < FP; ++b) {
      const cplx<T>* row = slice + b * F1;
      T rx = 0, ry = 0;
#pragma unroll
      for (int a = 0; a < FP; ++a) {
        const cplx<T> v = row[a];
        rx += a1[a] * v.x;
        ry += a1[a] * v.y;
      }
      px += a2[b] * rx;
      py += a2[b] * ry;
    }
    accx += wc * px;
    accy += wc * py;
  }
  return mk((double)accx, (double)accy);
}

// Footprint staging: each thread issues its loads 64 bytes at a time before writing LDS (lanes
// past the footprint load its first node again), so a block keeps several loads per thread in
// flight instead of waiting on each.
template <typename T> constexpr int stage_unroll() { return 64 / (int)sizeof(cplx<T>); }

// Stage field f's near footprint of a tile, (F1 x F2 x F3 nodes from (o1, o2, o3), periodic).
template <typename T, int F1, int F2, int F3>
__device__ __forceinline__ void stage_near(const GArgs& A, const cplx<T>* __restrict__ grid, int o1, int o2, int o3,
                                           int nfield, cplx<T>* lds) {
  constexpr int FSZ = F1 * F2 * F3, U = stage_unroll<T>();
  const int n = nfield * FSZ, nt = blockDim.x;
  for (int i0 = threadIdx.x; i0 < n; i0 += U * nt) {
    cplx<T> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = i0 + u * nt < n ? i0 + u * nt : 0;
      const int f = idx / FSZ, r = idx - f * FSZ;
      const int z = r / (F1 * F2), y = (r / F1) % F2, xx = r % F1;
      const int g1 = (o1 + xx) & (A.M1 - 1), g2 = (o2 + y) & (A.M2 - 1), g3 = (o3 + z) & (A.M3 - 1);
      v[u] = grid[f * A.fs + ((long)g3 * A.M2 + g2) * A.M1 + g1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * nt < n) lds[i0 + u * nt] = v[u];
  }
}

// Stage far field f's footprint of a tile (periodic in x1, x2; slices clamped to the slab:
// the clamped ones are never used by a stencil that lies in the slab).
template <typename T, int F1, int F2, int F3>
__device__ __forceinline__ void stage_far(const GArgs& A, const cplx<T>* __restrict__ far, int o1, int o2, int o3,
                                          cplx<T>* lds) {
  constexpr int FSZ = F1 * F2 * F3, U = stage_unroll<T>();
  const int nt = blockDim.x;
  for (int i0 = threadIdx.x; i0 < FSZ; i0 += U * nt) {
    cplx<T> v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int idx = i0 + u * nt < FSZ ? i0 + u * nt : 0;
      const int z = idx / (F1 * F2), y = (idx / F1) % F2, xx = idx % F1;
      const int g1 = (o1 + xx) & (A.Mf1 - 1), g2 = (o2 + y) & (A.Mf2 - 1);
      const int g3 = min(max(o3 + z, 0), A.S - 1);
      v[u] = far[((long)g3 * A.Mf2 + g2) * A.Mf1 + g1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + u * nt < FSZ) lds[i0 + u * nt] = v[u];
  }
}

// Near tiles: one block per tile, keys [0, nnear).  Stages the NF fields' footprint in LDS,
// then interpolates its targets (the next record prefetched); FP32 weights on the complex64
// path, FP64 add-back and phase, results in the caller's order.  A target whose stencil does
// not lie in the footprint (a rounding disagreement with the key pass) goes to the overflow list.
template <typename T, int NF, int TB1, int TB2, int TB3, int BS>
__global__ __launch_bounds__(BS) void k_gather3d_near(GArgs A, TileArgs B, const cplx<T>* __restrict__ grid,
                                                       const TRec* __restrict__ rec,
                                                       const uint32_t* __restrict__ hist,
                                                       const uint32_t* __restrict__ offs,
                                                       cplx<T>* __restrict__ out, uint8_t* __restrict__ flags,
                                                       uint32_t* __restrict__ ovf, uint32_t* __restrict__ novf) {
  constexpr int F1 = (1 << TB1) + 3, F2 = (1 << TB2) + 3, F3 = (1 << TB3) + 3, FSZ = F1 * F2 * F3;
  constexpr int NO = NOut<NF>::v;
  __shared__ cplx<T> lds[NF * FSZ];
  const int key = (int)blockIdx.x;
  const uint32_t cnt = hist[key];
  if (cnt == 0) return;
  const long start = offs[key];
  const int b1 = key % B.nt1, b2 = (key / B.nt1) % B.nt2, b3 = key / (B.nt1 * B.nt2);
  const int o1 = (b1 << TB1) - 1, o2 = (b2 << TB2) - 1, o3 = (b3 << TB3) - 1;
  stage_near<T, F1, F2, F3>(A, grid, o1, o2, o3, NF, lds);
  __syncthreads();
  const long end = start + (long)cnt;
  long j = start + threadIdx.x;
  TRec r{};
  if (j < end) r = rec[j];
  for (; j < end; j += BS) {
    TRec rn = r;
    if (j + BS < end) rn = rec[j + BS];
    Near3<T> s;
    near3_stencil<T>(A, r.x, r.y, r.z, s);
    const int l1 = (s.p1 - 1 - o1) & (A.M1 - 1), l2 = (s.p2 - 1 - o2) & (A.M2 - 1), l3 = (s.p3 - 1 - o3) & (A.M3 - 1);
    if (l1 > F1 - 4 || l2 > F2 - 4 || l3 > F3 - 4) {
      ovf[atomicAdd(novf, 1u)] = (uint32_t)j;
    } else {
      double2 L[NF];
      const cplx<T>* base = lds + (l3 * F2 + l2) * F1 + l1;
#pragma unroll
      for (int f = 0; f < NF; ++f) L[f] = lds_sum<T, F1, F2>(base + f * FSZ, s.w1, s.w2, s.w3);
      double2 res[NO];
      uint8_t fl = 0;
      near3_finish<T, NF>(A, r.x, r.y, r.z, s, L, res, fl);
      const long i = r.i;
#pragma unroll
      for (int o = 0; o < NO; ++o) store_out<T>(out, i * NO + o, res[o]);
      if (flags) flags[i] = fl;
    }
    r = rn;
  }
}

// Maxwell near tiles with few targets each: the fields are staged one after another into one
// footprint, each target's stencil sums kept in registers; up to BS targets per pass.
template <typename T, int NF, int TB1, int TB2, int TB3>
__global__ __launch_bounds__(256) void k_gather3d_near_fields(GArgs A, TileArgs B, const cplx<T>* __restrict__ grid,
                                                              const TRec* __restrict__ rec,
                                                              const uint32_t* __restrict__ hist,
                                                              const uint32_t* __restrict__ offs,
                                                              cplx<T>* __restrict__ out,
                                                              uint8_t* __restrict__ flags,
                                                              uint32_t* __restrict__ ovf,
                                                              uint32_t* __restrict__ novf) {
  constexpr int F1 = (1 << TB1) + 3, F2 = (1 << TB2) + 3, F3 = (1 << TB3) + 3, FSZ = F1 * F2 * F3;
  constexpr int NO = NOut<NF>::v;
  __shared__ cplx<T> lds[FSZ];
  const int key = (int)blockIdx.x;
  const uint32_t cnt = hist[key];
  if (cnt == 0) return;
  const long start = offs[key];
  const int b1 = key % B.nt1, b2 = (key / B.nt1) % B.nt2, b3 = key / (B.nt1 * B.nt2);
  const int o1 = (b1 << TB1) - 1, o2 = (b2 << TB2) - 1, o3 = (b3 << TB3) - 1;
  for (long c0 = 0; c0 < (long)cnt; c0 += blockDim.x) {
    const long j = start + c0 + threadIdx.x;
    const bool valid = c0 + (long)threadIdx.x < (long)cnt;
    TRec r{};
    Near3<T> s;
    bool miss = false;
    int l1 = 0, l2 = 0, l3 = 0;
    if (valid) {
      r = rec[j];
      near3_stencil<T>(A, r.x, r.y, r.z, s);
      l1 = (s.p1 - 1 - o1) & (A.M1 - 1);
      l2 = (s.p2 - 1 - o2) & (A.M2 - 1);
      l3 = (s.p3 - 1 - o3) & (A.M3 - 1);
      miss = l1 > F1 - 4 || l2 > F2 - 4 || l3 > F3 - 4;
    }
    double2 L[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      __syncthreads();   // the previous field's sums are done
      stage_near<T, F1, F2, F3>(A, grid + f * A.fs, o1, o2, o3, 1, lds);
      __syncthreads();
      if (valid && !miss) L[f] = lds_sum<T, F1, F2>(lds + (l3 * F2 + l2) * F1 + l1, s.w1, s.w2, s.w3);
    }
    if (!valid) continue;
    if (miss) {
      ovf[atomicAdd(novf, 1u)] = (uint32_t)j;
      continue;
    }
    double2 res[NO];
    uint8_t fl = 0;
    near3_finish<T, NF>(A, r.x, r.y, r.z, s, L, res, fl);
#pragma unroll
    for (int o = 0; o < NO; ++o) store_out<T>(out, (long)r.i * NO + o, res[o]);
    if (flags) flags[r.i] = fl;
  }
}

// Far tiles: one block per far key (keys nnear .. nnear + nfar - 1), and one more block for
// the last key (non-finite and out-of-slab targets: NaN).  The FP-point footprint of one field is
// staged at a time: for one field (G_d) once per tile; for the six Maxwell entries field by field
// for each pass of BS targets, whose sums stay in registers.
template <typename T, int NF, int FB1, int FB2, int FB3, int BS, int FP = far_points<T>()>
__global__ __launch_bounds__(BS) void k_gather3d_far(GArgs A, TileArgs B, const cplx<T>* __restrict__ grid,
                                                      const cplx<T>* __restrict__ far,
                                                      const TRec* __restrict__ rec,
                                                      const uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ offs,
                                                      cplx<T>* __restrict__ out, uint8_t* __restrict__ flags,
                                                      uint32_t* __restrict__ ovf, uint32_t* __restrict__ novf) {
  constexpr int F1 = (1 << FB1) + FP - 1, F2 = (1 << FB2) + FP - 1, F3 = (1 << FB3) + FP - 1;
  constexpr int LO = FP / 2 - 1;
  constexpr int NO = NOut<NF>::v;
  __shared__ cplx<T> lds[F1 * F2 * F3];
  const int key = B.nnear + (int)blockIdx.x;
  const uint32_t cnt = hist[key];
  if (cnt == 0) return;
  const long start = offs[key];
  if (key == B.nkeys - 1) {
    // non-finite coordinates (flag 8) and far targets beyond the slab (flags 2 and 4): NaN
    for (long j = start + threadIdx.x; j < start + (long)cnt; j += blockDim.x) {
      const TRec r = rec[j];
      const bool fin = isfinite(r.x) && isfinite(r.y) && isfinite(r.z);
#pragma unroll
      for (int o = 0; o < NO; ++o) store_out<T>(out, (long)r.i * NO + o, nan2());
      if (flags) flags[r.i] = fin ? 6 : 8;
    }
    return;
  }
  const int kk = key - B.nnear;
  const int b1 = kk % B.fnt1, b2 = (kk / B.fnt1) % B.fnt2, b3 = kk / (B.fnt1 * B.fnt2);
  const int o1 = (b1 << FB1) - LO, o2 = (b2 << FB2) - LO, o3 = (b3 << FB3) - LO;
  if (NO == 1) {
    stage_far<T, F1, F2, F3>(A, far, o1, o2, o3, lds);
    __syncthreads();
  }
  for (long c0 = 0; c0 < (long)cnt; c0 += BS) {
    const long j = start + c0 + threadIdx.x;
    const bool valid = c0 + (long)threadIdx.x < (long)cnt;
    TRec r{};
    Far3<T, FP> s;
    bool miss = false;
    int l1 = 0, l2 = 0, l3 = 0;
    if (valid) {
      r = rec[j];
      miss = !far3_stencil<T, FP>(A, r.x, r.y, r.z, s);
      l1 = (s.p1 - LO - o1) & (A.Mf1 - 1);
      l2 = (s.p2 - LO - o2) & (A.Mf2 - 1);
      l3 = s.s0 - LO - o3;
      miss = miss || l1 > F1 - FP || l2 > F2 - FP || l3 < 0 || l3 > F3 - FP;
    }
    double2 L[NO];
#pragma unroll
    for (int f = 0; f < NO; ++f) {
      if (NO > 1) {
        __syncthreads();   // the previous field's sums are done
        stage_far<T, F1, F2, F3>(A, far + f * A.ffs, o1, o2, o3, lds);
        __syncthreads();
      }
      if (valid && !miss) L[f] = lds_sump<T, F1, F2, FP>(lds + (l3 * F2 + l2) * F1 + l1, s.w1, s.w2, s.w3);
    }
    if (!valid) continue;
    if (miss) {
      ovf[atomicAdd(novf, 1u)] = (uint32_t)j;
      continue;
    }
    double2 res[NO];
    far3_finish<NO>(A, r.x, r.y, r.z, L, res);
#pragma unroll
    for (int o = 0; o < NO; ++o) store_out<T>(out, (long)r.i * NO + o, res[o]);
    if (flags) flags[r.i] = 2;
  }
}

constexpr int kFar8Threads = 512;   // 64 targets in flight per block

// DPP moves of a double within rows of 16 lanes (the control is a compile-time constant).
template <int CTRL>
__device__ __forceinline__ double dpp_d(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  return __hiloint2double(__builtin_amdgcn_update_dpp(0, hi, CTRL, 0xf, 0xf, false),
                          __builtin_amdgcn_update_dpp(0, lo, CTRL, 0xf, 0xf, false));
}
// Sum over each aligned group of 8 lanes, the total in every lane of the group: lane ^ 1, lane ^ 2
// (quad permutations), then the mirror within the half row (lane i with 7 - i) joins the quads.
__device__ __forceinline__ double sum8(double v) {
  v += dpp_d<0xB1>(v);    // quad_perm [1, 0, 3, 2]
  v += dpp_d<0x4E>(v);    // quad_perm [2, 3, 0, 1]
  v += dpp_d<0x141>(v);   // row_half_mirror
  return v;
}

// Complex128 far tiles, 8 lanes per target.  The LDS serves 128 bytes per clock (8 lanes of a
// 16-byte read); one target's 8-point stencil row is 8 contiguous nodes (128 bytes) of the
// staged footprint, so each group of 8 lanes reads one row per clock whatever its alignment,
// where one lane per target (random rows in every group of 8 lanes) waits on bank conflicts.
// Lane a of a group takes x1 node a of every row of the target's 8 x 8 x 8 stencil; the eight
// partial sums are joined by DPP moves.  Every lane of a group computes the target's stencil
// (the same record, so the group branches together).  Keys, footprints, overflow and results
// as k_gather3d_far; the Maxwell fields are staged one at a time for each pass of BS targets.
// PT = 7: a 7-point rule along x2 and x3 (the rows' first 7 nodes), 49 rows per target instead of
// 64, where the slab's spacing is fine enough for it (far7_ok).  Its error grows towards the
// lattice points, where the series' high modes matter most: sel = 1 takes only the tiles whose
// targets all lie at least kFar7Rmin from every lattice point (and the key of the targets outside
// the slab), sel = 2 only the others, on a grid of 2 c1 x 2 c2 x c3 blocks covering the c1 (c2)
// tiles next to x1 (x2) = 0 on either side and the first c3 slice tiles; sel = 0 every tile.
constexpr double kFar7Rmin = 0.8;
template <int NF, int FB1, int FB2, int FB3, int BS, int PT>
__global__ __launch_bounds__(BS) void k_gather3d_far8(GArgs A, TileArgs B, const double2* __restrict__ far,
                                                       const TRec* __restrict__ rec,
                                                       const uint32_t* __restrict__ hist,
                                                       const uint32_t* __restrict__ offs,
                                                       double2* __restrict__ out, uint8_t* __restrict__ flags,
                                                       uint32_t* __restrict__ ovf, uint32_t* __restrict__ novf,
                                                       int sel, int c1, int c2) {
  constexpr int FP = 8, LO = FP / 2 - 1;
  // x1 rows staged at a pitch of a multiple of 8 nodes (one node of padding): every row starts on
  // a 128-byte boundary, so the lane that reads node l1 + j of a row takes j = (a - l1) & 7, and the
  // eight lanes of a target read the 16-byte slots 0..7 of the LDS's 128-byte bank cycle in lane
  // order whatever the target's offset l1 (measured on gfx950: 116 against 87 bytes per clock per
  // CU for 8-lane groups at random offsets)
  constexpr int F1 = (1 << FB1) + FP, F2 = (1 << FB2) + FP - 1, F3 = (1 << FB3) + FP - 1;
  static_assert(F1 % 8 == 0, "x1 rows must start on 128-byte boundaries");
  constexpr int NO = NOut<NF>::v;
  constexpr int G = BS / 8;                  // targets in flight per block
  __shared__ double2 lds[F1 * F2 * F3];
  int key = B.nnear + (int)blockIdx.x;
  if (sel == 2) {
    const int i1 = (int)blockIdx.x % (2 * c1), i2 = ((int)blockIdx.x / (2 * c1)) % (2 * c2);
    const int i3 = (int)blockIdx.x / (4 * c1 * c2);
    const int t1 = i1 < c1 ? i1 : B.fnt1 - 2 * c1 + i1, t2 = i2 < c2 ? i2 : B.fnt2 - 2 * c2 + i2;
    key = B.nnear + (i3 * B.fnt2 + t2) * B.fnt1 + t1;
  }
  const uint32_t cnt = hist[key];
  if (cnt == 0) return;
  const long start = offs[key];
  if (key == B.nkeys - 1) {
    if (sel == 2) return;
    for (long j = start + threadIdx.x; j < start + (long)cnt; j += blockDim.x) {
      const TRec r = rec[j];
      const bool fin = isfinite(r.x) && isfinite(r.y) && isfinite(r.z);
#pragma unroll
      for (int o = 0; o < NO; ++o) out[(long)r.i * NO + o] = nan2();
      if (flags) flags[r.i] = fin ? 6 : 8;
    }
    return;
  }
  const int kk = key - B.nnear;
  const int b1 = kk % B.fnt1, b2 = (kk / B.fnt1) % B.fnt2, b3 = kk / (B.fnt1 * B.fnt2);
  if (sel != 0) {
    // the tile's targets: base nodes [lo, lo + 2^FB) per periodic axis (node i at x = i 2 pi / Mf,
    // periodic), base slices from b3 2^FB3 (|x3| >= c); their distance to the nearest lattice point
    const int lo1 = b1 << FB1, lo2 = b2 << FB2;
    const double d1 = min(lo1, A.Mf1 - lo1 - (1 << FB1)) * (2.0 * kPi / A.Mf1);
    const double d2 = min(lo2, A.Mf2 - lo2 - (1 << FB2)) * (2.0 * kPi / A.Mf2);
    const double z = fmax(A.c, A.fz0 + (double)(b3 << FB3) * A.hf);
    const bool close = d1 * d1 + d2 * d2 + z * z < kFar7Rmin * kFar7Rmin;
    if (close != (sel == 2)) return;
  }
  const int o1 = (b1 << FB1) - LO, o2 = (b2 << FB2) - LO, o3 = (b3 << FB3) - LO;
  const int g = (int)threadIdx.x >> 3, a = (int)threadIdx.x & 7;
  if (NO == 1) {
    stage_far<double, F1, F2, F3>(A, far, o1, o2, o3, lds);
    __syncthreads();
  }
  const long passes = NO == 1 ? 1 : ((long)cnt + BS - 1) / BS;
  for (long p = 0; p < passes; ++p) {
    const long t0 = NO == 1 ? 0 : p * BS, t1 = NO == 1 ? (long)cnt : std::min((long)cnt, t0 + BS);
#pragma unroll 1
    for (int f = 0; f < NO; ++f) {
      if (NO > 1) {
        __syncthreads();   // the previous field's reads are done
        stage_far<double, F1, F2, F3>(A, far + f * A.ffs, o1, o2, o3, lds);
        __syncthreads();
      }
#pragma unroll 1
      for (long t = t0 + g; t < t1; t += G) {
        const long j = start + t;
        const TRec r = rec[j];
        Far3<double, FP, PT> st;
        bool miss = !far3_stencil<double, FP, PT>(A, r.x, r.y, r.z, st);
        const int l1 = (st.p1 - LO - o1) & (A.Mf1 - 1);
        const int l2 = (st.p2 - LO - o2) & (A.Mf2 - 1);
        const int l3 = st.s0 - LO - o3;
        miss = miss || l1 > F1 - FP || l2 > F2 - FP || l3 < 0 || l3 > F3 - FP;
        if (miss) {
          if (f == 0 && a == 0) ovf[atomicAdd(novf, 1u)] = (uint32_t)j;
          continue;
        }
        // this lane's node of the x1 window and its weight (a select chain keeps the weights in
        // registers)
        const int jn = (a - l1) & 7;
        double w1a = st.w1[0];
#pragma unroll
        for (int m = 1; m < FP; ++m) w1a = jn == m ? st.w1[m] : w1a;
        const double2* node = lds + (l3 * F2 + l2) * F1 + l1 + jn;
        double ax = 0.0, ay = 0.0;
        double w3[PT];
#pragma unroll
        for (int m = 0; m < PT; ++m) w3[m] = st.w3[m];
        // all PT x PT rows unrolled: a wave has the reads of several slices in flight (measured
        // 0.71 -> 0.58 ms against a rolled slice loop; no spills at 512 threads per block)
#pragma unroll
        for (int c = 0; c < PT; ++c) {
          const double wc = w3[0];
#pragma unroll
          for (int m = 0; m < PT - 1; ++m) w3[m] = w3[m + 1];
          const double2* slice = node + c * (F2 * F1);
          double px = 0.0, py = 0.0;
#pragma unroll
          for (int b = 0; b < PT; ++b) {
            const double2 v = slice[b * F1];
            px = fma(st.w2[b], v.x, px);
            py = fma(st.w2[b], v.y, py);
          }
          ax = fma(wc, px, ax);
          ay = fma(wc, py, ay);
        }
        ax = sum8(w1a * ax);
        ay = sum8(w1a * ay);
        if (a == 0) {
          // the phase e^{i alpha.x'}; GG_13, GG_23 carry sgn(x3) (as far3_finish)
          double ps, pc;
          sincos(A.a1 * r.x + A.a2 * r.y, &ps, &pc);
          double2 v = cmul(mk(pc, ps), mk(ax, ay));
          if (NO == kMxO && f >= 4 && r.z < 0.0) v = cscale(v, -1.0);
          out[(long)r.i * NO + f] = v;
          if (flags && f == 0) flags[r.i] = 2;
        }
      }
    }
  }
}

// Targets the tiled kernels handed over (stencil outside the tile footprint): evaluated
// from global memory.  The count is read on the device.
template <typename T, int NF>
__global__ __launch_bounds__(256) void k_gather3d_overflow(GArgs A, const cplx<T>* __restrict__ grid,
                                                           const cplx<T>* __restrict__ far,
                                                           const TRec* __restrict__ rec,
                                                           const uint32_t* __restrict__ ovf,
                                                           const uint32_t* __restrict__ novf,
                                                           cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  constexpr int NO = NOut<NF>::v;
  const long n = *novf;
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
    const TRec r = rec[ovf[q]];
    const long i = r.i;
    double2 res[NO];
    uint8_t fl;
    eval3d_global<T, NF>(A, grid, far, r.x, r.y, r.z, res, fl);
#pragma unroll
    for (int o = 0; o < NO; ++o) store_out<T>(out, i * NO + o, res[o]);
    if (flags) flags[i] = fl;
  }
}

// 2D: G (Algorithm 2.1).
// i mod M for i in [-M, 2M): x1 node indices of the 2D grids, whose length M1 = 2^a r need not be a
// power of two
__device__ __forceinline__ int wrap_m(int i, int M) { return i < 0 ? i + M : (i >= M ? i - M : i); }

// 4 x 4 stencil sum of a 2D grid: rows[b] is the first element of stencil row b, i0 the
// first x1 node (periodic in x1).
template <typename T>
__device__ __forceinline__ double2 stencil2d_scalar(const cplx<T>* __restrict__ g, const long rows[4], int i0,
                                                    int M1, const T w1[4], const T w2[4]) {
  Acc<T> acc;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) acc.add(w2[b] * w1[a], g[rows[b] + wrap_m(i0 + a, M1)]);
  return acc.get();
}
template <typename T>
__device__ __forceinline__ double2 stencil2d(const cplx<T>* __restrict__ g, const long rows[4], int i0, int M1,
                                             const T w1[4], const T w2[4]) {
  return stencil2d_scalar<T>(g, rows, i0, M1, w1, w2);
}
// complex64 stencil rows.  Scattered targets make every load of a lane a cache lookup of its
// own, so a row of 4 nodes that does not wrap in x1 (32 contiguous bytes, 8-byte aligned) is
// read with two 16-byte loads instead of four 8-byte ones.
struct __attribute__((aligned(8))) F4a8 {
  float a, b, c, d;
};
// sum_a w[a] v[a] in a fixed order (every complex64 row sum takes it, so that the contiguous,
// the wrapped and the node-quad forms of a row give the same bits)
__device__ __forceinline__ float2 row4v(float2 v0, float2 v1, float2 v2, float2 v3, const float w[4]) {
  float re = w[0] * v0.x, im = w[0] * v0.y;
  re = fmaf(w[1], v1.x, re);
  im = fmaf(w[1], v1.y, im);
  re = fmaf(w[2], v2.x, re);
  im = fmaf(w[2], v2.y, im);
  re = fmaf(w[3], v3.x, re);
  im = fmaf(w[3], v3.y, im);
  return make_float2(re, im);
}
// sum_a w[a] r[a] over the 4 contiguous nodes at r
__device__ __forceinline__ float2 row4(const float2* __restrict__ r, const float w[4]) {
  const F4a8 lo = *reinterpret_cast<const F4a8*>(r);
  const F4a8 hi = *reinterpret_cast<const F4a8*>(r + 2);
  return row4v(make_float2(lo.a, lo.b), make_float2(lo.c, lo.d), make_float2(hi.a, hi.b), make_float2(hi.c, hi.d),
               w);
}

template <>
__device__ __forceinline__ double2 stencil2d<float>(const float2* __restrict__ g, const long rows[4], int i0, int M1,
                                                    const float w1[4], const float w2[4]) {
  float2 rs[4];
  if (i0 > M1 - 4) {
    // the row wraps in x1: four single loads, the same sums
#pragma unroll
    for (int b = 0; b < 4; ++b)
      rs[b] = row4v(g[rows[b] + i0], g[rows[b] + wrap_m(i0 + 1, M1)], g[rows[b] + wrap_m(i0 + 2, M1)],
                    g[rows[b] + wrap_m(i0 + 3, M1)], w1);
  } else {
#pragma unroll
    for (int b = 0; b < 4; ++b) rs[b] = row4(g + rows[b] + i0, w1);
  }
  float re = 0.f, im = 0.f;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    re = fmaf(w2[b], rs[b].x, re);
    im = fmaf(w2[b], rs[b].y, im);
  }
  return mk(re, im);
}

// complex64 node quads (q[4 node + a] = node + a along x1, wrapped): a stencil row is one
// 32-byte aligned run, so each row costs one memory sector instead of one or two, and rows
// that wrap in x1 need no special case.
__device__ __forceinline__ double2 stencil2d_quad(const float2* __restrict__ q, const long rows[4], int i0,
                                                  const float w1[4], const float w2[4]) {
  float re = 0.f, im = 0.f;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const float2 r = row4(q + (rows[b] + i0) * 4, w1);
    re = fmaf(w2[b], r.x, re);
    im = fmaf(w2[b], r.y, im);
  }
  return mk(re, im);
}

// NF fields interleaved per node (g[node * NF + f]): one 4 x 4 stencil gives all of them,
// and a stencil row of all fields is one contiguous run of 4 NF values.
template <typename T, int NF>
__device__ __forceinline__ void stencil2d_multi(const cplx<T>* __restrict__ g, const long rows[4], int i0, int M1,
                                                const T w1[4], const T w2[4], double2 L[NF]) {
  Acc<T> acc[NF];
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      const cplx<T>* q = g + (rows[b] + wrap_m(i0 + a, M1)) * NF;
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[f].add(w2[b] * w1[a], q[f]);
    }
#pragma unroll
  for (int f = 0; f < NF; ++f) L[f] = acc[f].get();
}
// complex64: a row that does not wrap in x1 is 4 NF float2 = 2 NF 16-byte loads
template <int NF>
__device__ __forceinline__ void stencil2d_multi_f32(const float2* __restrict__ g, const long rows[4], int i0, int M1,
                                                    const float w1[4], const float w2[4], double2 L[NF]) {
  if (i0 > M1 - 4) {
    stencil2d_multi<float, NF>(g, rows, i0, M1, w1, w2, L);
    return;
  }
  float re[NF], im[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) re[f] = im[f] = 0.f;
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const F4a8* r = reinterpret_cast<const F4a8*>(g + (rows[b] + i0) * NF);
    float v[8 * NF];
#pragma unroll
    for (int q = 0; q < 2 * NF; ++q) {
      const F4a8 t = r[q];
      v[4 * q] = t.a;
      v[4 * q + 1] = t.b;
      v[4 * q + 2] = t.c;
      v[4 * q + 3] = t.d;
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      float sr = w1[0] * v[2 * f], si = w1[0] * v[2 * f + 1];
#pragma unroll
      for (int a = 1; a < 4; ++a) {
        sr = fmaf(w1[a], v[2 * (a * NF + f)], sr);
        si = fmaf(w1[a], v[2 * (a * NF + f) + 1], si);
      }
      re[f] = fmaf(w2[b], sr, re[f]);
      im[f] = fmaf(w2[b], si, im[f]);
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) L[f] = mk(re[f], im[f]);
}
template <typename T, int NF>
__device__ __forceinline__ void stencil2d_fields(const cplx<T>* __restrict__ g, const long rows[4], int i0, int M1,
                                                 const T w1[4], const T w2[4], double2 L[NF]) {
  if constexpr (sizeof(T) == 4)
    stencil2d_multi_f32<NF>(g, rows, i0, M1, w1, w2, L);
  else
    stencil2d_multi<T, NF>(g, rows, i0, M1, w1, w2, L);
}

// Mark the wave's targets that lie in the cut-off ring: the wave's 64 consecutive targets own
// one word of the mask, which its first lane writes whole, so the mask needs neither clearing nor
// atomics.  Called by every lane of the wave (take false beyond the last target).
__device__ __forceinline__ void ring_mark(const GArgs& A, bool take, long i, long T_) {
  const unsigned long long m = __ballot(take);
  if (__lane_id() == 0 && i < T_) A.ring_mask[i >> 6] = m;
}

// Far branch of the 2D kinds (Algorithm 2.1 step 2b, the series (1.2) and its term-wise
// derivatives): the far slab (Mf1 modes, slices fz0 + s hf) interpolated with FP x FP nodes (8 on
// the complex128 path, 4 on the complex64 one), read in the plan's layout of it (A.far_layout:
// fields apart [f][s][i1], node quads, or fields interleaved per node [s][i1][f], as the near
// grid is read).  false when |x2| lies beyond the slab.
template <typename T, int NF>
__device__ __forceinline__ bool far2d_sum(const GArgs& A, const cplx<T>* __restrict__ far, double t, double z,
                                          double2 L[NF]) {
  constexpr int FP = far_points<T>(), LO = FP / 2 - 1;
  double s0, f2;
  if (!far_slice(A, z, s0, f2)) return false;
  T w1[FP], w2[FP];
  const double u = t * A.ihf1, p = floor(u);
  lagp<T, FP>((T)(u - p), w1);
  lagp<T, FP>((T)f2, w2);
  const int i0 = (int)p - LO;
  const long r0 = (long)s0 - LO;
  if constexpr (FP == 4) {
    // complex64: the near grid's row sums (one fixed order for the quads and the row-major slab,
    // so that single-instance plans and the batched call give the same bits)
    long rows[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) rows[b] = (r0 + b) * A.Mf1;
    const int j0 = i0 & (A.Mf1 - 1);
    if constexpr (NF == 1) {
      L[0] = A.far_layout == 1 ? stencil2d_quad(far, rows, j0, w1, w2) : stencil2d<T>(far, rows, j0, A.Mf1, w1, w2);
      return true;
    } else if (A.far_layout == 2) {
      stencil2d_fields<T, NF>(far, rows, j0, A.Mf1, w1, w2, L);
      return true;
    }
  }
  const long fstride = A.far_layout == 2 ? 1 : A.ffs, nstride = A.far_layout == 2 ? NF : 1;
  Acc<T> acc[NF];
#pragma unroll
  for (int b = 0; b < FP; ++b) {
    const long row = (r0 + b) * A.Mf1;
#pragma unroll
    for (int a = 0; a < FP; ++a) {
      const T w = w2[b] * w1[a];
      const long o = (row + ((i0 + a) & (A.Mf1 - 1))) * nstride;
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[f].add(w, far[f * fstride + o]);
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) L[f] = acc[f].get();
  return true;
}

// One target of Algorithm 2.1 step 2; returns whether it lies in the cut-off ring.
template <typename T>
__device__ __forceinline__ bool gather2d_one(const GArgs& A, const cplx<T>* __restrict__ grid,
                                             const cplx<T>* __restrict__ far, const double* __restrict__ x, long i,
                                             cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  const double x1 = x[2 * i], x2 = x[2 * i + 1];
  uint8_t fl = 0;
  bool in_ring = false;
  double2 res;
  if (!(isfinite(x1) && isfinite(x2))) {
    fl = 8;
    res = nan2();
  } else {
    double n1;
    const double t = reduce_cell(x1, n1);
    double ps, pc;
    sincos(A.a1 * x1, &ps, &pc);
    const double2 phase = mk(pc, ps);
    double2 Lt;
    if (fabs(x2) <= A.c) {
      T w1[4], w2[4];
      const double u = t * A.ih1, p = floor(u);
      lag4<T>((T)(u - p), w1);
      const int i0 = wrap_m((int)p - 1, A.M1);
      const double u2 = x2 * A.ih2, p2 = floor(u2);
      lag4<T>((T)(u2 - p2), w2);
      long rows[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) rows[b] = (long)(((int)p2 - 1 + b) & (A.M2 - 1)) * A.M1;
      if constexpr (sizeof(T) == 4) {
        if (A.quad) Lt = stencil2d_quad(grid, rows, i0, w1, w2);
        else Lt = stencil2d<T>(grid, rows, i0, A.M1, w1, w2);
      } else {
        Lt = stencil2d<T>(grid, rows, i0, A.M1, w1, w2);
      }
      const double r = sqrt(t * t + x2 * x2);
      if (r <= A.rmin || r == 0.0) {
        fl |= 1;
        Lt = nan2();
      } else if (r < 2.0 * A.eps) {
        // K_N = L_N + f1 - i alpha f2 = L_N - (1/2pi) ln r Y(r) (1 - i alpha t)
        const double s = -log(r) * cut_Y(r, A.eps) / (2.0 * kPi);
        in_ring = r > A.ring_lo;
        if (A.sing_order <= 1) {
          Lt = cadd(Lt, mk(s, -A.a1 * t * s));
        } else {
          // the higher-order factor P_m: 1 - i a t - (a^2/2) t^2 - (k^2/4) r^2 + i (a^3/6) t^3 + i (a k^2/4) t r^2
          const double a = A.a1, kk = 0.25 * A.k * A.k, r2 = t * t + x2 * x2;
          const double pr = 1.0 - 0.5 * a * a * t * t - kk * r2;
          double pim = -a * t;
          if (A.sing_order >= 3) pim += a * t * (a * a * t * t / 6.0 + kk * r2);
          Lt = cadd(Lt, mk(s * pr, s * pim));
        }
      } else if (r < A.ring_hi) {
        in_ring = r > A.ring_lo;
      }
    } else {
      fl |= 2;
      if (!far2d_sum<T, 1>(A, far, t, fabs(x2), &Lt)) {
        fl |= 4;
        Lt = nan2();
      }
    }
    res = cmul(phase, Lt);
  }
  store_out<T>(out, i, res);
  if (flags) flags[i] = fl;
  return in_ring;
}

// The cut-off ring (ring_interp): for the marked targets (r_lo < r < r_hi, every stencil node at
// least eps/2 from the lattice point) the stencil's sum of f Y over its
// nodes replaces f Y at the target, so that the result is the interpolant of K = L + f Y:
// out += e^{i alpha x1} (sum_ab w_a w_b (f Y)(node_ab) - (f Y)(target)), f the removed singular
// part of the plan's order and a node's position its offset (p1 h1, p2 h2) from the lattice
// point.  The correction is computed in FP64 on both paths (singular work next to the lattice
// point), as is the phase.  Each block takes
// kRingSpan consecutive targets: its first wave reads their mask words and collects the marked
// offsets in LDS, then all lanes correct them (kRingSpan targets per block: fewer, fuller blocks
// measured faster than small ones whose waves stay mostly idle).
template <typename C>
__device__ __forceinline__ cplx<C> cv(C re, C im) {
  cplx<C> v;
  v.x = re;
  v.y = im;
  return v;
}

template <typename C>
__device__ __forceinline__ C ring_log(C r) {
  if constexpr (sizeof(C) == 8) return log(r);
  else return __logf(r);
}

// Y_eps(r); in FP32 as S((2 eps - r)/eps) (S(1 - u) = 1 - S(u) for the symmetric Beta(9, 9)
// transition), which avoids the cancellation of 1 - S near the ring's outer edge.
template <typename C>
__device__ __forceinline__ C ring_cutY(const GArgs& A, C r) {
  if constexpr (sizeof(C) == 8) {
    return cut_Y(r, A.eps);
  } else {
    const float u = (2.0f * (float)A.eps - r) * (float)(1.0 / A.eps);
    if (u <= 0.0f) return 0.0f;
    if (u >= 1.0f) return 1.0f;
    const float binom[9] = {24310.0f, 19448.0f, 12376.0f, 6188.0f, 2380.0f, 680.0f, 136.0f, 17.0f, 1.0f};
    const float v = 1.0f - u;
    float uj = u * u * u;
    uj = uj * uj * uj;                                  // u^9
    float vp[9];
    vp[0] = 1.0f;
#pragma unroll
    for (int j = 1; j < 9; ++j) vp[j] = vp[j - 1] * v;  // v^0..v^8
    float sum = 0.0f;
#pragma unroll
    for (int j = 9; j <= 17; ++j) {
      sum += binom[j - 9] * uj * vp[17 - j];
      uj *= u;
    }
    return sum;
  }
}

template <typename C>
__device__ __forceinline__ cplx<C> fy_removed(const GArgs& A, C t, C z) {
  const C r2 = t * t + z * z;
  const C r = sqrt(r2);
  if (!(r < (C)(2.0 * A.eps)) || r2 == C(0)) return cv<C>(0, 0);
  const C s = -ring_log(r) * ring_cutY(A, r) / (C)(2.0 * kPi);
  const C a = (C)A.a1;
  C pr = 1, pim = -a * t;
  if (A.sing_order >= 2) {
    const C kk = (C)(0.25 * A.k * A.k);
    pr -= C(0.5) * a * a * t * t + kk * r2;
    if (A.sing_order >= 3) pim += a * t * (a * a * t * t / C(6) + kk * r2);
  }
  return cv<C>(s * pr, s * pim);
}

// The gradient's singular parts (Section 2.4.1) at cell point (t, z), zero beyond 2 eps:
// h_p = -(Y/2pi) [ -(k^2/2) x_p ln r + x_p/r^2 - i alpha t x_p/r^2 - (alpha^2/2) t^2 x_p/r^2 ],
// x_1 = t, x_2 = z.
template <typename C>
__device__ __forceinline__ void hgrad_at(const GArgs& A, C t, C z, cplx<C>& h1, cplx<C>& h2) {
  const C r2 = t * t + z * z;
  h1 = h2 = cv<C>(0, 0);
  if (!(r2 < (C)(4.0 * A.eps * A.eps)) || r2 == C(0)) return;
  const C r = sqrt(r2), ir2 = C(1) / r2;
  const C c = -ring_cutY(A, r) / (C)(2.0 * kPi);
  const C re = (C)(-0.5 * A.k * A.k) * ring_log(r) + ir2 - (C)(0.5 * A.a1 * A.a1) * t * t * ir2;
  const C im = (C)(-A.a1) * t * ir2;
  h1 = cv<C>(c * re * t, c * im * t);
  h2 = cv<C>(c * re * z, c * im * z);
}

// The second-derivative differences' singular parts (Section 2.4.2) at cell point (t, z), zero
// beyond 2 eps: h_pq = C Y [ s_pq - i alpha t s_pq ], C = (k1^2 - k2^2)/(2pi),
// s_11 = ln r/2 + t^2/(2r^2), s_12 = t z/(2r^2), s_22 = ln r/2 + z^2/(2r^2).
template <typename C>
__device__ __forceinline__ void hhess_at(const GArgs& A, C t, C z, cplx<C> h[3]) {
  const C r2 = t * t + z * z;
  h[0] = h[1] = h[2] = cv<C>(0, 0);
  if (!(r2 < (C)(4.0 * A.eps * A.eps)) || r2 == C(0)) return;
  const C r = sqrt(r2), ir2 = C(0.5) / r2, hl = C(0.5) * ring_log(r);
  const C Cy = (C)((A.k * A.k - A.k2 * A.k2) / (2.0 * kPi)) * ring_cutY(A, r);
  const C s11 = hl + t * t * ir2, s12 = t * z * ir2, s22 = hl + z * z * ir2;
  const C at = (C)(-A.a1) * t;
  h[0] = cv<C>(Cy * s11, Cy * at * s11);
  h[1] = cv<C>(Cy * s12, Cy * at * s12);
  h[2] = cv<C>(Cy * s22, Cy * at * s22);
}

constexpr int kRingWords = 256;                 // mask words per block of the ring pass (one per thread)
constexpr int kRingSpan = 64 * kRingWords;      // targets per block
static_assert(kRingSpan <= 65536, "k_ring2d keeps 16-bit offsets in LDS");

template <typename T, int NF>
__global__ __launch_bounds__(256) void k_ring2d(GArgs A, const double* __restrict__ x, long T_,
                                                cplx<T>* __restrict__ out) {
  __shared__ uint32_t s_n;
  __shared__ uint16_t s_off[kRingSpan];
  const int tid = threadIdx.x;
  if (tid == 0) s_n = 0;
  __syncthreads();
  const long base = (long)blockIdx.x * kRingSpan;
  if (tid < kRingWords) {
    const long w = (base >> 6) + tid;
    unsigned long long m = w < (T_ + 63) >> 6 ? A.ring_mask[w] : 0ull;
    if (m) {
      uint32_t pos = atomicAdd(&s_n, (uint32_t)__popcll(m));
      while (m) {
        const int b = __ffsll((long long)m) - 1;
        s_off[pos++] = (uint16_t)(tid * 64 + b);
        m &= m - 1;
      }
    }
  }
  __syncthreads();
  const uint32_t n = s_n;
  for (uint32_t j = tid; j < n; j += 256) {
    const long i = base + s_off[j];
    const double x1 = x[2 * i], x2 = x[2 * i + 1];
    double n1;
    const double t = reduce_cell(x1, n1);
    const double u = t * A.ih1, p = floor(u), u2 = x2 * A.ih2, p2 = floor(u2);
    // the singular part near the origin in FP64 on both paths (only the grid values are complex64)
    double w1[4], w2[4];
    lag4<double>(u - p, w1);
    lag4<double>(u2 - p2, w2);
    // NF = 1: f Y of the 2D G; NF = 2: the gradient's h1, h2; NF = 3: h_11, h_12, h_22
    double2 acc[NF], at[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = mk(0.0, 0.0);
    for (int b = 0; b < 4; ++b) {
      const double zn = (p2 - 1.0 + b) * A.h2;
      double2 row[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) row[f] = mk(0.0, 0.0);
      for (int a = 0; a < 4; ++a) {
        const double tn = (p - 1.0 + a) * A.h1;
        double2 v[NF];
        if constexpr (NF == 1) v[0] = fy_removed<double>(A, tn, zn);
        else if constexpr (NF == 2) hgrad_at<double>(A, tn, zn, v[0], v[1]);
        else hhess_at<double>(A, tn, zn, v);
#pragma unroll
        for (int f = 0; f < NF; ++f) row[f] = mk(fma(w1[a], v[f].x, row[f].x), fma(w1[a], v[f].y, row[f].y));
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[f] = mk(fma(w2[b], row[f].x, acc[f].x), fma(w2[b], row[f].y, acc[f].y));
    }
    if constexpr (NF == 1) at[0] = fy_removed<double>(A, t, x2);
    else if constexpr (NF == 2) hgrad_at<double>(A, t, x2, at[0], at[1]);
    else hhess_at<double>(A, t, x2, at);
    double ps, pc;
    sincos(A.a1 * x1, &ps, &pc);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double2 corr = cmul(mk(pc, ps), mk(acc[f].x - at[f].x, acc[f].y - at[f].y));
      const cplx<T> o = out[i * NF + f];
      store_out<T>(out, i * NF + f, mk((double)o.x + corr.x, (double)o.y + corr.y));
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather2d(GArgs A, const cplx<T>* __restrict__ grid,
                                                  const cplx<T>* __restrict__ far, const double* __restrict__ x,
                                                  long T_, cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in_ring = i < T_ && gather2d_one<T>(A, grid, far, x, i, out, flags);
  if (A.ring_mask) ring_mark(A, in_ring, i, T_);
}

// One target of the 2D gradient (Section 2.4.1): both fields interpolated with one
// stencil, the singular parts h1, h2 added back in FP64 inside 2 eps, the phase
// e^{i alpha x1}; beyond c the far slab of the differentiated series, the x2 field times
// sgn(x2).  grid holds the two near fields interleaved per node, far the two far fields one
// after the other.  out[2i] = dG/dx1, out[2i+1] = dG/dx2.  Returns whether the target lies in
// the cut-off ring (when the plan marks them).
template <typename T>
__device__ __forceinline__ bool gather2d_grad_one(const GArgs& A, const cplx<T>* __restrict__ grid,
                                                  const cplx<T>* __restrict__ far, const double* __restrict__ x,
                                                  long i, cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  const double x1 = x[2 * i], x2 = x[2 * i + 1];
  uint8_t fl = 0;
  bool in_ring = false;
  double2 d1, d2;
  if (!(isfinite(x1) && isfinite(x2))) {
    fl = 8;
    d1 = d2 = nan2();
  } else {
    double n1;
    const double t = reduce_cell(x1, n1);
    double ps, pc;
    sincos(A.a1 * x1, &ps, &pc);
    const double2 phase = mk(pc, ps);
    double2 L[2];
    if (fabs(x2) <= A.c) {
      T w1[4], w2[4];
      const double u = t * A.ih1, p = floor(u);
      lag4<T>((T)(u - p), w1);
      const int i0 = wrap_m((int)p - 1, A.M1);
      const double u2 = x2 * A.ih2, p2 = floor(u2);
      lag4<T>((T)(u2 - p2), w2);
      long rows[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) rows[b] = (long)(((int)p2 - 1 + b) & (A.M2 - 1)) * A.M1;
      stencil2d_fields<T, 2>(grid, rows, i0, A.M1, w1, w2, L);
      const double r2 = t * t + x2 * x2;
      if (r2 <= A.rmin * A.rmin || r2 == 0.0) {
        fl |= 1;
        L[0] = L[1] = nan2();
      } else {
        if (r2 < 4.0 * A.eps * A.eps) {
          double2 h1, h2;
          hgrad_at(A, t, x2, h1, h2);
          L[0] = cadd(L[0], h1);
          L[1] = cadd(L[1], h2);
        }
        if (A.ring_mask) {
          const double r = sqrt(r2);
          in_ring = r > A.ring_lo && r < A.ring_hi;
        }
      }
    } else {
      fl |= 2;
      if (!far2d_sum<T, 2>(A, far, t, fabs(x2), L)) {
        fl |= 4;
        L[0] = L[1] = nan2();
      } else if (x2 < 0.0) {
        L[1] = cscale(L[1], -1.0);
      }
    }
    d1 = cmul(phase, L[0]);
    d2 = cmul(phase, L[1]);
  }
  store_out<T>(out, 2 * i, d1);
  store_out<T>(out, 2 * i + 1, d2);
  if (flags) flags[i] = fl;
  return in_ring;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather2d_grad(GArgs A, const cplx<T>* __restrict__ grid,
                                                       const cplx<T>* __restrict__ far, const double* __restrict__ x,
                                                       long T_, cplx<T>* __restrict__ out,
                                                       uint8_t* __restrict__ flags) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in_ring = i < T_ && gather2d_grad_one<T>(A, grid, far, x, i, out, flags);
  if (A.ring_mask) ring_mark(A, in_ring, i, T_);
}

// One target of the second-derivative differences (Section 2.4.2): three fields with one
// stencil, h_pq added back in FP64 inside 2 eps, the phase e^{i alpha x1}; beyond c the far
// slab of the twice-differentiated series, the 12 field times sgn(x2).  grid holds the three
// near fields interleaved per node, far the three far fields one after the other.
// out[3i + p] = d_p d_q G_k1 - d_p d_q G_k2, pq = 11, 12, 22.
template <typename T>
__device__ __forceinline__ bool gather2d_hess_one(const GArgs& A, const cplx<T>* __restrict__ grid,
                                                  const cplx<T>* __restrict__ far, const double* __restrict__ x,
                                                  long i, cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  const double x1 = x[2 * i], x2 = x[2 * i + 1];
  uint8_t fl = 0;
  bool in_ring = false;
  double2 L[3];
  if (!(isfinite(x1) && isfinite(x2))) {
    fl = 8;
    L[0] = L[1] = L[2] = nan2();
  } else {
    double n1;
    const double t = reduce_cell(x1, n1);
    double ps, pc;
    sincos(A.a1 * x1, &ps, &pc);
    const double2 phase = mk(pc, ps);
    if (fabs(x2) <= A.c) {
      T w1[4], w2[4];
      const double u = t * A.ih1, p = floor(u);
      lag4<T>((T)(u - p), w1);
      const int i0 = wrap_m((int)p - 1, A.M1);
      const double u2 = x2 * A.ih2, p2 = floor(u2);
      lag4<T>((T)(u2 - p2), w2);
      long rows[4];
#pragma unroll
      for (int b = 0; b < 4; ++b) rows[b] = (long)(((int)p2 - 1 + b) & (A.M2 - 1)) * A.M1;
      stencil2d_fields<T, 3>(grid, rows, i0, A.M1, w1, w2, L);
      const double r2 = t * t + x2 * x2;
      if (r2 <= A.rmin * A.rmin || r2 == 0.0) {
        fl |= 1;
        L[0] = L[1] = L[2] = nan2();
      } else {
        if (r2 < 4.0 * A.eps * A.eps) {
          double2 h[3];
          hhess_at(A, t, x2, h);
#pragma unroll
          for (int f = 0; f < 3; ++f) L[f] = cadd(L[f], h[f]);
        }
        if (A.ring_mask) {
          const double r = sqrt(r2);
          in_ring = r > A.ring_lo && r < A.ring_hi;
        }
      }
    } else {
      fl |= 2;
      if (!far2d_sum<T, 3>(A, far, t, fabs(x2), L)) {
        fl |= 4;
        L[0] = L[1] = L[2] = nan2();
      } else if (x2 < 0.0) {
        L[1] = cscale(L[1], -1.0);
      }
    }
#pragma unroll
    for (int f = 0; f < 3; ++f) L[f] = cmul(phase, L[f]);
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) store_out<T>(out, 3 * i + f, L[f]);
  if (flags) flags[i] = fl;
  return in_ring;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather2d_hess(GArgs A, const cplx<T>* __restrict__ grid,
                                                       const cplx<T>* __restrict__ far, const double* __restrict__ x,
                                                       long T_, cplx<T>* __restrict__ out,
                                                       uint8_t* __restrict__ flags) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in_ring = i < T_ && gather2d_hess_one<T>(A, grid, far, x, i, out, flags);
  if (A.ring_mask) ring_mark(A, in_ring, i, T_);
}

// Many 2D instances in one launch: instance i owns blocks [blk0_i, blk0_{i+1}) and
// targets [t0_i, t1_i) of the concatenated target array.
struct GatherInst {
  GArgs A;
  long off, foff;     // first element of the instance's near grid / far slab
  long t0, t1;
  long blk0;
};

template <typename T>
__global__ __launch_bounds__(256) void k_gather2d_multi(const GatherInst* __restrict__ inst, int n_inst,
                                                        const cplx<T>* __restrict__ grid,
                                                        const cplx<T>* __restrict__ far,
                                                        const double* __restrict__ x, cplx<T>* __restrict__ out,
                                                        uint8_t* __restrict__ flags) {
  int lo = 0, hi = n_inst - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].blk0 <= (long)blockIdx.x) lo = mid;
    else hi = mid - 1;
  }
  const GatherInst I = inst[lo];
  const long i = I.t0 + ((long)blockIdx.x - I.blk0) * blockDim.x + threadIdx.x;
  if (i < I.t1) gather2d_one<T>(I.A, grid + I.off, far + I.foff, x, i, out, flags);
}

// ---------------------------------------------------------------------------
// Target binning (counting sort by grid tile): key pass with an atomic rank
// inside each tile, one-block exclusive scan, scatter into tile order.
// ---------------------------------------------------------------------------
struct BinArgs {
  double c, ih1, ih2, ih3;
  double fz0, ihf, ihf1, ihf2;   // far slab: first slice, reciprocal spacings
  int M1, M2, M3, S, Mf1, Mf2;
  int fp;                        // far-slab interpolation points per axis
  TileArgs t;
};

// The tile of a target: the tile of its stencil's base node (near: the 4-point base on the
// near grid; far: the 8-point base on the far slab), the same arithmetic as the gathers'.
__device__ __forceinline__ uint32_t tile_key(const BinArgs& B, double x1, double x2, double x3) {
  if (!(isfinite(x1) && isfinite(x2) && isfinite(x3))) return B.t.nkeys - 1;
  double n;
  const double t1 = reduce_cell(x1, n), t2 = reduce_cell(x2, n);
  if (fabs(x3) <= B.c) {
    const int b1 = (((int)floor(t1 * B.ih1)) & (B.M1 - 1)) >> B.t.tb1;
    const int b2 = (((int)floor(t2 * B.ih2)) & (B.M2 - 1)) >> B.t.tb2;
    const int b3 = (((int)floor(x3 * B.ih3)) & (B.M3 - 1)) >> B.t.tb3;
    return (uint32_t)((b3 * B.t.nt2 + b2) * B.t.nt1 + b1);
  }
  double s0 = floor((fabs(x3) - B.fz0) * B.ihf);
  if (!(s0 <= B.S - 1 - B.fp / 2)) return B.t.nkeys - 1;
  s0 = fmax(s0, (double)(B.fp / 2 - 1));
  const int b1 = (((int)floor(t1 * B.ihf1)) & (B.Mf1 - 1)) >> B.t.ftb1;
  const int b2 = (((int)floor(t2 * B.ihf2)) & (B.Mf2 - 1)) >> B.t.ftb2;
  const int b3 = (int)s0 >> B.t.ftb3;
  return (uint32_t)(B.t.nnear + (b3 * B.t.fnt2 + b2) * B.t.fnt1 + b1);
}

__global__ void k_zero_u32(uint32_t* __restrict__ p, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0u;
}

__global__ __launch_bounds__(256) void k_bin_key(BinArgs B, const double* __restrict__ x, long T_,
                                                 uint32_t* __restrict__ hist, uint2* __restrict__ keyrank) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T_) return;
  const uint32_t key = tile_key(B, x[3 * i], x[3 * i + 1], x[3 * i + 2]);
  const uint32_t r = atomicAdd(&hist[key], 1u);
  keyrank[i] = make_uint2(key, r);
}

// exclusive scan of hist[0..n) into offs[0..n) with one block of 1024 threads.  Up to 32 x 1024 keys:
// thread t reads keys t + 1024 j (coalesced, all loads issued first) and the block scans one row of
// 1024 keys at a time (64-lane shuffle scans, then the 16 wave totals), carrying the running total
// from row to row.  More keys: each thread sums a contiguous segment, the block scans the segment
// sums and each thread writes its segment's prefixes.
constexpr int kScanRows = 32;
__global__ __launch_bounds__(1024) void k_bin_scan(const uint32_t* __restrict__ hist, uint32_t* __restrict__ offs,
                                                   int n) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x;
  if (n <= kScanRows * 1024) {
    const int lane = t & 63, w = t >> 6, rows = (n + 1023) / 1024;
    uint32_t v[kScanRows];
#pragma unroll
    for (int j = 0; j < kScanRows; ++j) {
      const int i = t + j * 1024;
      v[j] = j < rows && i < n ? hist[i] : 0u;
    }
    uint32_t carry = 0;
#pragma unroll
    for (int j = 0; j < kScanRows; ++j) {
      if (j < rows) {   // uniform over the block
        uint32_t x = v[j];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
          const uint32_t y = __shfl_up(x, d, 64);
          if (lane >= d) x += y;
        }
        if (lane == 63) part[w] = x;   // wave totals
        __syncthreads();
        if (w == 0) {
          uint32_t q = lane < 16 ? part[lane] : 0u;
#pragma unroll
          for (int d = 1; d < 16; d <<= 1) {
            const uint32_t y = __shfl_up(q, d, 64);
            if (lane >= d) q += y;
          }
          if (lane < 16) part[lane] = q;   // inclusive prefixes of the wave totals
        }
        __syncthreads();
        const int i = t + j * 1024;
        if (i < n) offs[i] = carry + (w > 0 ? part[w - 1] : 0u) + x - v[j];
        carry += part[15];
        __syncthreads();
      }
    }
    return;
  }
  const int per = (n + 1023) / 1024;
  const int lo = min(n, t * per), hi = min(n, lo + per);
  uint32_t s = 0;
  for (int i = lo; i < hi; ++i) s += hist[i];
  part[t] = s;
  __syncthreads();
  for (int d = 1; d < 1024; d <<= 1) {
    uint32_t v = t >= d ? part[t - d] : 0u;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  uint32_t run = part[t] - s;
  for (int i = lo; i < hi; ++i) {
    offs[i] = run;
    run += hist[i];
  }
}

__global__ __launch_bounds__(256) void k_bin_scatter(const double* __restrict__ x, const uint2* __restrict__ keyrank,
                                                     const uint32_t* __restrict__ offs, long T_,
                                                     TRec* __restrict__ rec) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T_) return;
  const uint2 kr = keyrank[i];
  const long pos = (long)offs[kr.x] + kr.y;
  TRec r;
  r.x = x[3 * i];
  r.y = x[3 * i + 1];
  r.z = x[3 * i + 2];
  r.i = (uint32_t)i;
  r.pad = 0u;
  rec[pos] = r;
}

// Binning without per-target global atomics (used when the key count fits an
// LDS histogram): each of kBinBlocks blocks takes a contiguous chunk of targets,
//  (1) counts its tile keys in LDS and writes the counts to cnt[block][key],
//  (2) k_bin_colscan turns cnt into per-(block, key) exclusive prefixes over the
//      blocks and per-key totals,
//  (3) k_bin_scan gives per-key offsets, and
//  (4) each block re-derives its keys and scatters its targets to
//      offs[key] + cnt[block][key] + (LDS-atomic rank within the block).
constexpr int kBinBlocks = 256;
constexpr int kMinPerTile = 1500;   // targets per tile below which the larger tiles are used
constexpr int kMaxPerFieldTile = 512;   // Maxwell: targets per 16 x 16 x 8 tile below which fields are staged one by one
constexpr int kBinUnroll = 8;
constexpr int kBinLdsKeys = 32768;   // 128 KiB of LDS: one 1024-thread block per CU

template <int KEYS>
__global__ __launch_bounds__(1024) void k_bin_count(BinArgs B, const double* __restrict__ x, long T_, long chunk,
                                                    uint32_t* __restrict__ cnt) {
  __shared__ uint32_t h[KEYS];
  const int nk = B.t.nkeys;
  for (int k = threadIdx.x; k < nk; k += blockDim.x) h[k] = 0u;
  __syncthreads();
  const long lo = (long)blockIdx.x * chunk, hi = min(T_, lo + chunk);
  // kBinUnroll independent coordinate loads in flight per thread
  for (long i0 = lo + threadIdx.x; i0 < hi; i0 += (long)kBinUnroll * blockDim.x) {
    double a[kBinUnroll], b[kBinUnroll], c[kBinUnroll];
#pragma unroll
    for (int u = 0; u < kBinUnroll; ++u) {
      const long i = i0 + (long)u * blockDim.x;
      if (i < hi) {
        a[u] = x[3 * i];
        b[u] = x[3 * i + 1];
        c[u] = x[3 * i + 2];
      }
    }
#pragma unroll
    for (int u = 0; u < kBinUnroll; ++u)
      if (i0 + (long)u * blockDim.x < hi) atomicAdd(&h[tile_key(B, a[u], b[u], c[u])], 1u);
  }
  __syncthreads();
  uint32_t* row = cnt + (long)blockIdx.x * nk;
  for (int k = threadIdx.x; k < nk; k += blockDim.x) row[k] = h[k];
}

// 64 keys per block; 16 groups of 64 threads each scan a sixteenth of the blocks.
constexpr int kColGroups = 16;
__global__ __launch_bounds__(64 * kColGroups) void k_bin_colscan(uint32_t* __restrict__ cnt, int nk, int nblk,
                                                                 uint32_t* __restrict__ total) {
  __shared__ uint32_t part[kColGroups][64];
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int k = blockIdx.x * 64 + lane;
  const int per = (nblk + kColGroups - 1) / kColGroups, b0 = grp * per, b1 = min(nblk, b0 + per);
  uint32_t s = 0;
  if (k < nk)
    for (int b = b0; b < b1; ++b) s += cnt[(long)b * nk + k];
  part[grp][lane] = s;
  __syncthreads();
  uint32_t run = 0;
  for (int g = 0; g < grp; ++g) run += part[g][lane];
  if (k < nk) {
    for (int b = b0; b < b1; ++b) {
      const long o = (long)b * nk + k;
      const uint32_t c = cnt[o];
      cnt[o] = run;
      run += c;
    }
    if (grp == kColGroups - 1) total[k] = run;
  }
}

template <int KEYS>
__global__ __launch_bounds__(1024) void k_bin_place(BinArgs B, const double* __restrict__ x, long T_, long chunk,
                                                    const uint32_t* __restrict__ cnt,
                                                    const uint32_t* __restrict__ offs, TRec* __restrict__ rec) {
  __shared__ uint32_t cur[KEYS];
  const int nk = B.t.nkeys;
  const uint32_t* row = cnt + (long)blockIdx.x * nk;
  for (int k = threadIdx.x; k < nk; k += blockDim.x) cur[k] = offs[k] + row[k];
  __syncthreads();
  const long lo = (long)blockIdx.x * chunk, hi = min(T_, lo + chunk);
  for (long i0 = lo + threadIdx.x; i0 < hi; i0 += (long)kBinUnroll * blockDim.x) {
    double a[kBinUnroll], b[kBinUnroll], c[kBinUnroll];
#pragma unroll
    for (int u = 0; u < kBinUnroll; ++u) {
      const long i = i0 + (long)u * blockDim.x;
      if (i < hi) {
        a[u] = x[3 * i];
        b[u] = x[3 * i + 1];
        c[u] = x[3 * i + 2];
      }
    }
#pragma unroll
    for (int u = 0; u < kBinUnroll; ++u) {
      const long i = i0 + (long)u * blockDim.x;
      if (i < hi) {
        const long pos = atomicAdd(&cur[tile_key(B, a[u], b[u], c[u])], 1u);
        TRec r;
        r.x = a[u];
        r.y = b[u];
        r.z = c[u];
        r.i = (uint32_t)i;
        r.pad = 0u;
        rec[pos] = r;
      }
    }
  }
}

// [field][node] -> [node][field] for the near grid and the far slab of the 2D derivative
// kinds (one thread per output element: coalesced writes, NF coalesced read streams).
template <typename T>
__global__ __launch_bounds__(256) void k_interleave(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                    long n, int nf) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n * nf) return;
  const long node = e / nf;
  const int f = (int)(e - node * nf);
  out[e] = in[f * n + node];
}

// Node quads of a complex64 2D grid or far slab with rows of M1 nodes: q[4 e + a] = in[row of e,
// x1 index of e + a, wrapped] (one thread per output value: coalesced writes).
__global__ __launch_bounds__(256) void k_quads(const float2* __restrict__ in, float2* __restrict__ q, long n,
                                               int M1) {
  const long v = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= 4 * n) return;
  const long e = v >> 2;
  const int a = (int)(v & 3);
  const long row = e / M1;
  const int i1 = (int)(e - row * M1);
  q[v] = in[row * M1 + wrap_m(i1 + a, M1)];
}

enum GatherMode { kGatherAll = 0, kBinOnly = 1, kGatherBinned = 2 };

template <typename T>
GArgs make_gargs(const Plan& P, int smooth) {
  GArgs A;
  A.k = P.last_k;
  A.k2 = P.last_k2;
  A.a1 = P.last_a1;
  A.a2 = P.last_a2;
  A.c = P.p.c;
  A.c_tilde = P.p.c_tilde;
  A.eps = P.p.eps;
  A.rmin = P.p.lattice_rmin;
  A.M1 = P.M1;
  A.M2 = P.M2;
  A.M3 = P.M3;
  A.h1 = kPi / (P.M1 / 2);
  if (P.dim == 2) {
    A.h2 = P.p.c_tilde / (P.M2 / 2);
    A.h3 = 0.0;
  } else {
    A.h2 = kPi / (P.M2 / 2);
    A.h3 = P.p.c_tilde / (P.M3 / 2);
  }
  A.ih1 = 1.0 / A.h1;
  A.ih2 = 1.0 / A.h2;
  A.ih3 = A.h3 > 0.0 ? 1.0 / A.h3 : 0.0;
  A.hf = P.hf;
  A.ihf = 1.0 / P.hf;
  A.fz0 = P.fz0;
  A.S = P.S;
  A.fp = P.fp;
  A.Mf1 = P.Mf1;
  A.Mf2 = P.Mf2;
  A.ihf1 = P.Mf1 / (2.0 * kPi);
  A.ihf2 = P.Mf2 / (2.0 * kPi);
  A.fs = (long)P.ncell;
  A.ffs = (long)P.nfar;
  A.smooth = smooth;
  A.sing_order = P.p.sing_order;
  A.quad = P.dim == 2 && P.nf == 1 && P.gridI != nullptr;
  A.far_layout = (P.dim == 2 && P.farI != nullptr) ? (P.nf == 1 ? 1 : 2) : 0;
  A.ring_mask = nullptr;
  // the ring zone r_lo < r < r_hi: r_hi = 2 eps + 2 sqrt(2) h, beyond which every stencil node has
  // Y = 0; r_lo = max(eps, eps/2 + 2 sqrt(2) h) keeps every node at least eps/2 from the lattice point
  const double reach = 2.0 * sqrt(2.0) * fmax(A.h1, A.h2);
  A.ring_lo = fmax(A.eps, 0.5 * A.eps + reach);
  A.ring_hi = 2.0 * A.eps + reach;
  return A;
}

template <typename T>
hipError_t gather2d_impl(Plan& P, GArgs& A, const double* x, int64_t T_, void* out, uint8_t* flags) {
  const auto* g = static_cast<const cplx<T>*>(P.grid);
  const auto* f = static_cast<const cplx<T>*>(P.far);
  const auto* gi = static_cast<const cplx<T>*>(P.gridI);
  if (A.far_layout) f = static_cast<const cplx<T>*>(P.farI);
  auto* o = static_cast<cplx<T>*>(out);
  const dim3 grid((unsigned)((T_ + 255) / 256));
  if (P.p.ring_interp) {
    hipError_t e = ensure_ring_scratch(P, T_);
    if (e != hipSuccess) return e;
    A.ring_mask = P.ts.ring_mask;
  }
  {
    KernelTimer t(P, QPGF_T_GATHER);   // the gather alone; the ring pass has its own timer
    if (P.nf == 2)
      hipLaunchKernelGGL(k_gather2d_grad<T>, grid, dim3(256), 0, P.stream, A, gi, f, x, (long)T_, o, flags);
    else if (P.nf == 3)
      hipLaunchKernelGGL(k_gather2d_hess<T>, grid, dim3(256), 0, P.stream, A, gi, f, x, (long)T_, o, flags);
    else
      hipLaunchKernelGGL(k_gather2d<T>, grid, dim3(256), 0, P.stream, A, A.quad ? gi : g, f, x, (long)T_, o, flags);
  }
  if (P.p.ring_interp) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    KernelTimer tr(P, QPGF_T_RING);
    const dim3 nb((unsigned)((T_ + kRingSpan - 1) / kRingSpan));
    if (P.nf == 3)
      hipLaunchKernelGGL((k_ring2d<T, 3>), nb, dim3(256), 0, P.stream, A, x, (long)T_, o);
    else if (P.nf == 2)
      hipLaunchKernelGGL((k_ring2d<T, 2>), nb, dim3(256), 0, P.stream, A, x, (long)T_, o);
    else
      hipLaunchKernelGGL((k_ring2d<T, 1>), nb, dim3(256), 0, P.stream, A, x, (long)T_, o);
  }
  return hipGetLastError();
}

// Tile configuration of a binned 3D call (kept in the plan between the binning and the gather).
struct TileCfg {
  TileArgs t;
  bool big, fields, far_big;
};
static_assert(sizeof(TileCfg) <= sizeof(int) * 24, "Plan::bt holds the tile configuration");

template <typename T, int NF>
hipError_t gather3d_impl(Plan& P, const GArgs& A, const double* x, int64_t T_, void* out, uint8_t* flags,
                         int mode, hipStream_t bin_stream) {
  const auto* g = static_cast<const cplx<T>*>(P.grid);
  const auto* f = static_cast<const cplx<T>*>(P.far);
  auto* o = static_cast<cplx<T>*>(out);
  const dim3 grid((unsigned)((T_ + 255) / 256));
  if (A.smooth || P.bin_min_targets < 0 || T_ < P.bin_min_targets) {
    KernelTimer t(P, QPGF_T_GATHER);
    hipLaunchKernelGGL((k_gather3d<T, NF>), grid, dim3(256), 0, P.stream, A, g, f, x, (long)T_, o, flags);
    return hipGetLastError();
  }
  BinArgs B;
  B.c = A.c;
  B.ih1 = A.ih1;
  B.ih2 = A.ih2;
  B.ih3 = A.ih3;
  B.fz0 = A.fz0;
  B.ihf = A.ihf;
  B.ihf1 = A.ihf1;
  B.ihf2 = A.ihf2;
  B.M1 = P.M1;
  B.M2 = P.M2;
  B.M3 = P.M3;
  B.S = P.S;
  B.Mf1 = P.Mf1;
  B.Mf2 = P.Mf2;
  B.fp = P.fp;
  if (P.fp != far_points<T>()) return hipErrorInvalidValue;
  // Near tiles.  One field: 16 x 16 x 8 nodes (several 256-thread blocks per CU, so one
  // block's staging overlaps the others' interpolation), or, when that leaves fewer than
  // kMinPerTile targets per tile on average (fine grids), 32 x 32 x 8 (complex64, 108 KiB,
  // 1024 threads) or 32 x 16 x 8 (complex128, 117 KiB, 512 threads).  Maxwell: 8 x 8 x 4
  // (complex64) or 8 x 4 x 4 (complex128) with every field staged (47 / 60 KiB for seven
  // fields), or 16 x 16 x 8 staged field by field when the tiles hold few targets.
  // Far tiles (one field staged at a time): complex128 (8-point footprints) 8 x 8 x 8 nodes
  // (53 KiB), or 16 x 8 x 8 (81 KiB) when the 8-node tiles' keys would not fit the LDS histograms
  // of the binning; complex64 (4-point footprints) 16 x 16 x 8 (19 x 19 x 11 nodes, 31 KiB: fewer
  // keys, so longer runs of the binning's record writes, and less halo per owned node).
  // Must match the instantiations below.
  TileCfg C{};
  TileArgs& Tl = C.t;
  auto set_near = [&](int a, int b, int c) {
    Tl.tb1 = a;
    Tl.tb2 = b;
    Tl.tb3 = c;
    Tl.nt1 = std::max(1, P.M1 >> a);
    Tl.nt2 = std::max(1, P.M2 >> b);
    Tl.nt3n = std::max(1, P.M3 >> c);
    Tl.nnear = Tl.nt1 * Tl.nt2 * Tl.nt3n;
  };
  hipError_t e = hipSuccess;
  if (mode == kGatherBinned) {
    // the configuration launch_bin3d used for these targets
    if (P.bt_T != T_ || P.bt_x != x) return hipErrorInvalidValue;
    std::memcpy(&C, P.bt, sizeof C);
  } else {
    if (NF > 1) {
      set_near(4, 4, 3);
      C.fields = T_ < (int64_t)kMaxPerFieldTile * Tl.nnear;
      if (!C.fields) set_near(3, sizeof(T) == 8 ? 2 : 3, 2);
    } else {
      set_near(4, 4, 3);
      if (T_ < (int64_t)kMinPerTile * Tl.nnear) {
        C.big = true;
        set_near(5, sizeof(T) == 8 ? 4 : 5, 3);
      }
    }
    auto set_far = [&](bool big) {
      C.far_big = big;
      Tl.ftb1 = big ? 4 : 3;
      Tl.ftb2 = big && sizeof(T) == 4 ? 4 : 3;
      Tl.ftb3 = 3;
      Tl.fnt1 = std::max(1, P.Mf1 >> Tl.ftb1);
      Tl.fnt2 = std::max(1, P.Mf2 >> Tl.ftb2);
      Tl.fnt3 = ((P.S - 1 - P.fp / 2) >> Tl.ftb3) + 1;
      Tl.nfar = Tl.fnt1 * Tl.fnt2 * Tl.fnt3;
      Tl.nkeys = Tl.nnear + Tl.nfar + 1;
    };
    // complex128: 8-node far tiles (two blocks per CU) unless their keys would overflow the LDS
    // histograms; complex64 (4-point stencils, small footprints): 16 x 16 x 8 far tiles
    set_far(sizeof(T) == 4);
    if (Tl.nkeys > kBinLdsKeys) set_far(true);
    e = ensure_bin_scratch(P, T_, Tl.nkeys);
    if (e != hipSuccess) return e;
    std::memcpy(P.bt, &C, sizeof C);
    P.bt_T = T_;
    P.bt_x = x;
  }
  B.t = Tl;
  TRec* rec = reinterpret_cast<TRec*>(P.ts.bin_rec);
  const bool lds_bins = Tl.nkeys <= kBinLdsKeys;
  const long chunk = (T_ + kBinBlocks - 1) / kBinBlocks;
  const hipStream_t bs = bin_stream ? bin_stream : P.stream;
  if (mode != kGatherBinned) {
    {
      KernelTimer t(P, QPGF_T_BIN, bs);
      hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, bs, P.ts.bin_novf, 1L);
      if (lds_bins) {
        // LDS histogram sized to the key count (small ones leave LDS to kernels running beside)
#define QPGF_BIN_COUNT(K_)                                                                                     \
  hipLaunchKernelGGL(k_bin_count<K_>, dim3(kBinBlocks), dim3(1024), 0, bs, B, x, (long)T_, chunk, P.ts.bin_cnt)
        if (Tl.nkeys <= 4096) QPGF_BIN_COUNT(4096);
        else if (Tl.nkeys <= 16384) QPGF_BIN_COUNT(16384);
        else if (Tl.nkeys <= 20480) QPGF_BIN_COUNT(20480);
        else if (Tl.nkeys <= 24576) QPGF_BIN_COUNT(24576);
        else QPGF_BIN_COUNT(kBinLdsKeys);
#undef QPGF_BIN_COUNT
        hipLaunchKernelGGL(k_bin_colscan, dim3((Tl.nkeys + 63) / 64), dim3(64 * kColGroups), 0, bs, P.ts.bin_cnt,
                           Tl.nkeys, kBinBlocks, P.ts.bin_hist);
      } else {
        // large key spaces: one global atomic rank per target
        hipLaunchKernelGGL(k_zero_u32, dim3((Tl.nkeys + 255) / 256), dim3(256), 0, bs, P.ts.bin_hist,
                           (long)Tl.nkeys);
        hipLaunchKernelGGL(k_bin_key, grid, dim3(256), 0, bs, B, x, (long)T_, P.ts.bin_hist, P.ts.bin_keyrank);
      }
      hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, bs, P.ts.bin_hist, P.ts.bin_offs, Tl.nkeys);
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    {
      KernelTimer t(P, QPGF_T_BIN_PLACE, bs);
#define QPGF_BIN_PLACE(K_)                                                                                     \
  hipLaunchKernelGGL(k_bin_place<K_>, dim3(kBinBlocks), dim3(1024), 0, bs, B, x, (long)T_, chunk, P.ts.bin_cnt, \
                     P.ts.bin_offs, rec)
      // the LDS histograms are sized to the key count, so that the binning's blocks leave LDS to the
      // preparation's kernels running beside them on the plan's stream
      if (lds_bins && Tl.nkeys <= 4096) QPGF_BIN_PLACE(4096);
      else if (lds_bins && Tl.nkeys <= 16384) QPGF_BIN_PLACE(16384);
      else if (lds_bins && Tl.nkeys <= 20480) QPGF_BIN_PLACE(20480);
      else if (lds_bins && Tl.nkeys <= 24576) QPGF_BIN_PLACE(24576);
      else if (lds_bins) QPGF_BIN_PLACE(kBinLdsKeys);
      else
        hipLaunchKernelGGL(k_bin_scatter, grid, dim3(256), 0, bs, x, P.ts.bin_keyrank, P.ts.bin_offs, (long)T_, rec);
#undef QPGF_BIN_PLACE
      e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  if (mode == kBinOnly) return hipSuccess;
  {
    const dim3 tn(Tl.nnear), tf(Tl.nfar + 1);
#define QPGF_NEAR(A1_, A2_, A3_, BS_)                                                                             \
  hipLaunchKernelGGL((k_gather3d_near<T, NF, A1_, A2_, A3_, BS_>), tn, dim3(BS_), 0, P.stream, A, Tl, g, rec,     \
                     P.ts.bin_hist, P.ts.bin_offs, o, flags, P.ts.bin_ovf, P.ts.bin_novf)
#define QPGF_FAR(A1_, A2_, A3_)                                                                                    \
  hipLaunchKernelGGL((k_gather3d_far<T, NF, A1_, A2_, A3_, 256>), tf, dim3(256), 0, P.stream, A, Tl, g, f, rec,    \
                     P.ts.bin_hist, P.ts.bin_offs, o, flags, P.ts.bin_ovf, P.ts.bin_novf)
#define QPGF_FAR8G(A1_, A2_, A3_, BS_, PT_, SEL_, G_, C1_, C2_)                                                  \
  hipLaunchKernelGGL((k_gather3d_far8<NF, A1_, A2_, A3_, BS_, PT_>), G_, dim3(BS_), 0, P.stream, A, Tl, f, rec,      \
                     P.ts.bin_hist, P.ts.bin_offs, o, flags, P.ts.bin_ovf, P.ts.bin_novf, SEL_, C1_, C2_)
#define QPGF_FAR8(A1_, A2_, A3_, BS_, PT_, SEL_) QPGF_FAR8G(A1_, A2_, A3_, BS_, PT_, SEL_, tf, 0, 0)
    // far tiles first (more targets and work each), then the near tiles
    {
      KernelTimer t(P, QPGF_T_GATHER_FAR);
      if constexpr (sizeof(T) == 8) {
        if (NF == 1 && far7_ok(P)) {
          // 7 points along x2 and x3 away from the lattice points; 8 in the few tiles next to them,
          // on a grid of those tiles only (c1, c2 tiles on either side of x = 0, c3 slice tiles)
          const int fb1 = C.far_big ? 4 : 3;
          const double h1 = 2.0 * kPi / P.Mf1, h2 = 2.0 * kPi / P.Mf2;
          const int c1 = std::min((int)std::ceil(kFar7Rmin / (h1 * (1 << fb1))), Tl.fnt1 / 2);
          const int c2 = std::min((int)std::ceil(kFar7Rmin / (h2 * 8)), Tl.fnt2 / 2);
          const int c3 = std::min((int)std::ceil((kFar7Rmin - P.fz0) / (P.hf * 8)) + 1, Tl.fnt3);
          const dim3 t8((unsigned)std::max(1, 4 * c1 * c2 * c3));
          if (!C.far_big) {
            QPGF_FAR8(3, 3, 3, kFar8Threads, 7, 1);
            if (c1 > 0 && c2 > 0 && c3 > 0) QPGF_FAR8G(3, 3, 3, kFar8Threads, 8, 2, t8, c1, c2);
          } else {
            QPGF_FAR8(4, 3, 3, kFar8Threads, 7, 1);
            if (c1 > 0 && c2 > 0 && c3 > 0) QPGF_FAR8G(4, 3, 3, kFar8Threads, 8, 2, t8, c1, c2);
          }
        } else {
          if (!C.far_big) QPGF_FAR8(3, 3, 3, kFar8Threads, 8, 0);
          else QPGF_FAR8(4, 3, 3, kFar8Threads, 8, 0);
        }
      } else {
        if (!C.far_big) QPGF_FAR(3, 3, 3);
        else QPGF_FAR(4, 4, 3);
      }
    }
    KernelTimer t(P, QPGF_T_GATHER);
    if constexpr (NF > 1) {
      if (C.fields)
        hipLaunchKernelGGL((k_gather3d_near_fields<T, NF, 4, 4, 3>), tn, dim3(256), 0, P.stream, A, Tl, g, rec,
                           P.ts.bin_hist, P.ts.bin_offs, o, flags, P.ts.bin_ovf, P.ts.bin_novf);
      else if constexpr (sizeof(T) == 8) QPGF_NEAR(3, 2, 2, 256);
      else QPGF_NEAR(3, 3, 2, 256);
    } else if (C.big) {
      if constexpr (sizeof(T) == 8) QPGF_NEAR(5, 4, 3, 512);
      else QPGF_NEAR(5, 5, 3, 1024);
    } else {
      QPGF_NEAR(4, 4, 3, 256);
    }
#undef QPGF_NEAR
#undef QPGF_FAR
#undef QPGF_FAR8
#undef QPGF_FAR8G
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  KernelTimer t(P, QPGF_T_OVERFLOW);
  hipLaunchKernelGGL((k_gather3d_overflow<T, NF>), dim3(64), dim3(256), 0, P.stream, A, g, f, rec, P.ts.bin_ovf,
                     P.ts.bin_novf, o, flags);
  return hipGetLastError();
}

template <typename T>
hipError_t gather_impl(Plan& P, const double* x, int64_t T_, void* out, uint8_t* flags, int smooth = 0,
                       int mode = kGatherAll, hipStream_t bin_stream = nullptr) {
  GArgs A = make_gargs<T>(P, smooth);
  if (P.dim == 2) return gather2d_impl<T>(P, A, x, T_, out, flags);
  if (P.nf == kMxF) return gather3d_impl<T, kMxF>(P, A, x, T_, out, flags, mode, bin_stream);
  if (P.nf == kMxT) return gather3d_impl<T, kMxT>(P, A, x, T_, out, flags, mode, bin_stream);
  return gather3d_impl<T, 1>(P, A, x, T_, out, flags, mode, bin_stream);
}

}  // namespace

// The complex128 G_d far gather may take 7 points along x2 and x3 (the 8-point rule's error
// constant 1.1e-3 against 2.4e-3 for 7 points, at one power of the spacing less): propagating
// terms (q <= k) then leave 2.4e-3 (k h)^7 <= 2e-11 for k h <= 0.07 along x2 (h = 2 pi / Mf2) and
// along x3 (h = hf), and the evanescent terms that reach c leave about 1e-11 at the geometry's
// floors (512 modes, hf <= 1/64).  Only on the automatic geometry (no far_m / far_h override).
bool far7_ok(const Plan& P) {
  if (P.p.far_m != 0 || P.p.far_h != 0.0 || P.dim != 3) return false;
  const double k = std::max(P.last_k, P.last_k2);
  return k * P.hf <= 0.07 && k * (2.0 * kPi / P.Mf2) <= 0.07;
}

// The near grid's and the far slab's copies in the gather's layout (rows of M1 and Mf1 nodes).
hipError_t launch_interleave2d(Plan& P) {
  if (P.dim != 2 || !P.gridI || !P.farI) return hipErrorInvalidValue;
  const void* src[2] = {P.grid, P.far};
  void* dst[2] = {P.gridI, P.farI};
  const long n[2] = {(long)P.ncell, (long)P.nfar};
  const int m1[2] = {P.M1, P.Mf1}, nf[2] = {P.nf, P.nfo};
  for (int w = 0; w < 2; ++w) {
    if (P.nf == 1) {
      // complex64 G: node quads
      if (P.esize != 8) return hipErrorInvalidValue;
      hipLaunchKernelGGL(k_quads, dim3((unsigned)((4 * n[w] + 255) / 256)), dim3(256), 0, P.stream,
                         static_cast<const float2*>(src[w]), static_cast<float2*>(dst[w]), n[w], m1[w]);
    } else {
      const long tot = n[w] * nf[w];
      if (P.esize == 16)
        hipLaunchKernelGGL(k_interleave<double>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, P.stream,
                           static_cast<const double2*>(src[w]), static_cast<double2*>(dst[w]), n[w], nf[w]);
      else
        hipLaunchKernelGGL(k_interleave<float>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, P.stream,
                           static_cast<const float2*>(src[w]), static_cast<float2*>(dst[w]), n[w], nf[w]);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t ensure_ring_scratch(Plan& P, int64_t T_) {
  TargetScratch& S = P.ts;
  const int64_t words = (T_ + 63) / 64;
  if (words <= S.ring_words) return hipSuccess;
  if (S.ext) return hipErrorInvalidValue;   // callers check the capacity first
  if (S.ring_mask) (void)hipFree(S.ring_mask);
  S.ring_mask = nullptr;
  S.ring_words = 0;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&S.ring_mask), (size_t)words * sizeof(unsigned long long));
  if (e != hipSuccess) return e;
  S.ring_words = words;
  return hipSuccess;
}

hipError_t ensure_bin_scratch(Plan& P, int64_t T_, int nkeys) {
  TargetScratch& S = P.ts;
  if (S.ext) {
    const bool fits = T_ <= S.bin_cap && nkeys <= S.bin_keycap && (nkeys > kBinLdsKeys || nkeys <= S.bin_cntkeys);
    return fits ? hipSuccess : hipErrorInvalidValue;
  }
  if (T_ > S.bin_cap) {
    for (void* q : {(void*)S.bin_keyrank, (void*)S.bin_rec, (void*)S.bin_ovf})
      if (q) (void)hipFree(q);
    S.bin_keyrank = nullptr;
    S.bin_rec = nullptr;
    S.bin_ovf = nullptr;
    S.bin_cap = 0;
    hipError_t e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.bin_keyrank), (size_t)T_ * sizeof(uint2))) != hipSuccess) return e;
    if ((e = hipMalloc(&S.bin_rec, (size_t)T_ * sizeof(TRec))) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.bin_ovf), (size_t)T_ * sizeof(uint32_t))) != hipSuccess) return e;
    S.bin_cap = T_;
  }
  if (nkeys > S.bin_keycap) {
    for (void* q : {(void*)S.bin_hist, (void*)S.bin_offs, (void*)S.bin_cnt})
      if (q) (void)hipFree(q);
    S.bin_hist = nullptr;
    S.bin_offs = nullptr;
    S.bin_cnt = nullptr;
    S.bin_keycap = 0;
    S.bin_cntkeys = 0;
    hipError_t e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.bin_hist), (size_t)nkeys * sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.bin_offs), (size_t)nkeys * sizeof(uint32_t))) != hipSuccess) return e;
    if (!S.bin_novf && (e = hipMalloc(reinterpret_cast<void**>(&S.bin_novf), sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&S.bin_cnt), (size_t)nkeys * kBinBlocks * sizeof(uint32_t))) !=
        hipSuccess)
      return e;
    S.bin_keycap = nkeys;
    S.bin_cntkeys = nkeys;
  }
  return hipSuccess;
}

void free_target_scratch(TargetScratch& S) {
  if (!S.ext) {
    for (void* q : {(void*)S.ring_mask, (void*)S.bin_keyrank, S.bin_rec, (void*)S.bin_hist, (void*)S.bin_offs,
                    (void*)S.bin_cnt, (void*)S.bin_ovf, (void*)S.bin_novf})
      if (q) (void)hipFree(q);
  }
  S = TargetScratch{};
}

// The tile choices of gather3d_impl, taken at their largest key counts: the near tiles of the
// kind (Maxwell: the smaller of its two configurations), the 8-node far tiles unless their keys
// overflow the LDS histograms, else the larger far tiles.  Any slab up to (Mf1, Mf2, S) has at
// most this many keys: with the small far tiles the keys stay within kBinLdsKeys.
int bin_keys_bound(const Plan& P, int Mf1, int Mf2, int S, int fp) {
  if (P.dim != 3) return 0;
  const bool c64 = P.esize == 8;
  auto tiles = [](int n, int b) { return std::max(1, n >> b); };
  long nnear = (long)tiles(P.M1, 4) * tiles(P.M2, 4) * tiles(P.M3, 3);
  if (P.nf > 1) nnear = std::max(nnear, (long)tiles(P.M1, 3) * tiles(P.M2, c64 ? 3 : 2) * tiles(P.M3, 2));
  const long fnt3 = ((S - 1 - fp / 2) >> 3) + 1;
  const long small = (long)tiles(Mf1, 3) * tiles(Mf2, 3) * fnt3;
  const long big = (long)tiles(Mf1, 4) * tiles(Mf2, c64 ? 4 : 3) * fnt3;
  const long ks = nnear + small + 1;
  return (int)(ks <= kBinLdsKeys ? ks : std::max<long>(kBinLdsKeys, nnear + big + 1));
}

size_t carve_target_scratch(const Plan& P, char* base, int64_t T_, int nkeys, TargetScratch& S) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* p = base ? base + off : nullptr;
    off += (bytes + 255) & ~(size_t)255;
    return p;
  };
  TargetScratch t;
  t.ext = true;
  if (P.dim == 3) {
    const int cntkeys = std::min(nkeys, kBinLdsKeys);
    t.bin_cap = T_;
    t.bin_keycap = nkeys;
    t.bin_cntkeys = cntkeys;
    t.bin_keyrank = reinterpret_cast<uint2*>(take((size_t)T_ * sizeof(uint2)));
    t.bin_rec = take((size_t)T_ * sizeof(TRec));
    t.bin_ovf = reinterpret_cast<uint32_t*>(take((size_t)T_ * sizeof(uint32_t)));
    t.bin_hist = reinterpret_cast<uint32_t*>(take((size_t)nkeys * sizeof(uint32_t)));
    t.bin_offs = reinterpret_cast<uint32_t*>(take((size_t)nkeys * sizeof(uint32_t)));
    t.bin_novf = reinterpret_cast<uint32_t*>(take(sizeof(uint32_t)));
    t.bin_cnt = reinterpret_cast<uint32_t*>(take((size_t)cntkeys * kBinBlocks * sizeof(uint32_t)));
  } else if (P.p.ring_interp) {
    t.ring_words = (T_ + 63) / 64;
    t.ring_mask = reinterpret_cast<unsigned long long*>(take((size_t)t.ring_words * sizeof(unsigned long long)));
  }
  if (base) S = t;
  return off;
}

void gather_inst_2d(const Plan& P, double k, double a, int M1, const FarGeom& fg, long off, long foff, long t0,
                    long t1, long blk0, void* dst) {
  GatherInst I;
  GArgs& A = I.A;
  A = make_gargs<double>(P, 0);
  A.k = k;
  A.k2 = 0.0;
  A.a1 = a;
  A.a2 = 0.0;
  A.M1 = M1;
  A.h1 = kPi / (M1 / 2);
  A.ih1 = 1.0 / A.h1;
  A.Mf1 = fg.Mf1;
  A.ihf1 = fg.Mf1 / (2.0 * kPi);
  A.S = fg.S;
  A.hf = fg.hf;
  A.ihf = 1.0 / fg.hf;
  A.fp = fg.P;
  A.fz0 = P.p.c - (fg.P / 2 - 1) * fg.hf;
  A.fs = (long)M1 * P.M2;
  A.ffs = (long)fg.Mf1 * fg.S;
  A.quad = 0;   // the batched graph keeps the instances' grids row by row (node quads of all
                // instances cost more than they save: four times the grids no longer stay in L2)
  A.far_layout = 0;
  A.ring_mask = nullptr;
  A.ring_lo = A.ring_hi = 0.0;
  I.off = off;
  I.foff = foff;
  I.t0 = t0;
  I.t1 = t1;
  I.blk0 = blk0;
  *static_cast<GatherInst*>(dst) = I;
}
size_t gather_inst_size() { return sizeof(GatherInst); }

hipError_t launch_gather2d_multi(Plan& P, const void* dinst, int n_inst, long nblocks, const void* grid,
                                 const void* far, const double* x, void* out, uint8_t* flags) {
  const auto* in = static_cast<const GatherInst*>(dinst);
  if (P.p.prec == QPGF_C128)
    hipLaunchKernelGGL(k_gather2d_multi<double>, dim3((unsigned)nblocks), dim3(256), 0, P.stream, in, n_inst,
                       static_cast<const double2*>(grid), static_cast<const double2*>(far), x,
                       static_cast<double2*>(out), flags);
  else
    hipLaunchKernelGGL(k_gather2d_multi<float>, dim3((unsigned)nblocks), dim3(256), 0, P.stream, in, n_inst,
                       static_cast<const float2*>(grid), static_cast<const float2*>(far), x,
                       static_cast<float2*>(out), flags);
  return hipGetLastError();
}

hipError_t launch_gather_smooth(Plan& P, const double* x, int64_t T_, void* out) {
  if (T_ <= 0) return hipSuccess;
  return P.p.prec == QPGF_C128 ? gather_impl<double>(P, x, T_, out, nullptr, 1)
                               : gather_impl<float>(P, x, T_, out, nullptr, 1);
}

hipError_t launch_gather(Plan& P, const double* x, int64_t T_, void* out, uint8_t* flags) {
  if (T_ <= 0) return hipSuccess;
  return P.p.prec == QPGF_C128 ? gather_impl<double>(P, x, T_, out, flags) : gather_impl<float>(P, x, T_, out, flags);
}

bool gather_uses_bins(const Plan& P, int64_t T_) {
  return P.dim == 3 && P.bin_min_targets >= 0 && T_ >= P.bin_min_targets;
}

hipError_t launch_bin3d(Plan& P, const double* x, int64_t T_, hipStream_t stream) {
  if (!gather_uses_bins(P, T_)) return hipErrorInvalidValue;
  return P.p.prec == QPGF_C128 ? gather_impl<double>(P, x, T_, nullptr, nullptr, 0, kBinOnly, stream)
                               : gather_impl<float>(P, x, T_, nullptr, nullptr, 0, kBinOnly, stream);
}

hipError_t launch_gather_binned(Plan& P, const double* x, int64_t T_, void* out, uint8_t* flags) {
  if (!gather_uses_bins(P, T_)) return hipErrorInvalidValue;
  return P.p.prec == QPGF_C128 ? gather_impl<double>(P, x, T_, out, flags, 0, kGatherBinned)
                               : gather_impl<float>(P, x, T_, out, flags, 0, kGatherBinned);
}

}  // namespace qpgf
