// Calculation step of Algorithms 2.1 / 3.1 / 4.1 for many targets: reduce each
// target to the period cell (step 2c), branch on |x_t| <= c (step 2b),
// interpolate the near grid with the tensor-product 4-point Lagrange rule
// (16 / 64 nodes, step 2d), add back the removed singular part in FP64 and apply
// the quasi-periodic phase (steps 2e-2f; Algorithm 4.1 steps 2e-2i).  Far
// targets interpolate the far-slab grid of the eigenfunction series.
#include <algorithm>

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
  double hf, ihf;          // far-slab spacing and its reciprocal
  int S;                   // far-slab slices
  long fs, ffs;            // field strides (near, far)
  int smooth;              // 1: return the interpolated smooth part L_N only (near branch)
  int sing_order;          // 2D G: degree of the removed Taylor factor of the log singularity (1..3)
  int quad;                // 2D G, complex64: grid and far are node quads (4 x1-neighbours per node)
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

// Stencil sum over global memory: field f, base nodes p1, p2 (periodic) and p3
// (near: periodic slice index; far: far-slab slice s0 >= 1).
template <typename T, int NF>
struct GlobalFetch {
  const cplx<T>* grid;
  const cplx<T>* far;
  long fs, ffs;
  int M1, M2, M3;
  __device__ void operator()(bool near, int p1, int p2, int p3, const T w1[4], const T w2[4], const T w3[4],
                             double2 L[NF]) const {
    const cplx<T>* g = near ? grid : far;
    const long st = near ? fs : ffs;
    Acc<T> acc[NF];
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const long i3 = near ? (long)((p3 - 1 + c) & (M3 - 1)) : (long)(p3 - 1 + c);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const long row = (i3 * M2 + ((p2 - 1 + b) & (M2 - 1))) * (long)M1;
        const T wcb = w3[c] * w2[b];
#pragma unroll
        for (int a = 0; a < 4; ++a) {
          const T w = wcb * w1[a];
          const long o = row + ((p1 - 1 + a) & (M1 - 1));
#pragma unroll
          for (int f = 0; f < NF; ++f) acc[f].add(w, g[f * st + o]);
        }
      }
    }
#pragma unroll
    for (int f = 0; f < NF; ++f) L[f] = acc[f].get();
  }
};

// The steps of eval3d_target (below) split in two, for kernels that compute the
// stencil sums between them (k_gather3d_fields): the stencil of one target
// (Algorithm 3.1 / 4.1 step 2: cell reduction, branch, base nodes and the three
// 4-point weight sets), and the finish from the sums to the result.  The
// single-function form stays for the other kernels, where it compiles to far
// fewer registers with six fields.
template <typename T>
struct Stencil3 {
  double t1, t2, n1, n2;
  bool near;
  int p1, p2, p3;
  T w1[4], w2[4], w3[4];
};

// false: the result is NaN without a stencil sum (non-finite input, beyond the
// far slab, or a far target when only the smooth part is asked for); res, fl set.
template <typename T, int NO>
__device__ __forceinline__ bool stencil3d(const GArgs& A, double x1, double x2, double x3, Stencil3<T>& s,
                                          double2* res, uint8_t& fl) {
  fl = 0;
  if (!(isfinite(x1) && isfinite(x2) && isfinite(x3))) {
    fl = 8;
#pragma unroll
    for (int o = 0; o < NO; ++o) res[o] = nan2();
    return false;
  }
  s.t1 = reduce_cell(x1, s.n1);
  s.t2 = reduce_cell(x2, s.n2);
  const double u1 = s.t1 * A.ih1, q1 = floor(u1);
  lag4<T>((T)(u1 - q1), s.w1);
  const double u2 = s.t2 * A.ih2, q2 = floor(u2);
  lag4<T>((T)(u2 - q2), s.w2);
  s.p1 = (int)q1;
  s.p2 = (int)q2;
  s.near = fabs(x3) <= A.c;
  if (s.near) {
    const double u = x3 * A.ih3, q = floor(u);
    lag4<T>((T)(u - q), s.w3);
    s.p3 = (int)q;
    return true;
  }
  fl |= 2;
  if (A.smooth) {
#pragma unroll
    for (int o = 0; o < NO; ++o) res[o] = nan2();
    return false;
  }
  const double v = (fabs(x3) - (A.c - A.hf)) * A.ihf;
  double s0 = floor(v);
  if (s0 > A.S - 3) {
    fl |= 4;
#pragma unroll
    for (int o = 0; o < NO; ++o) res[o] = nan2();
    return false;
  }
  s0 = fmax(s0, 1.0);
  lag4<T>((T)(v - s0), s.w3);
  s.p3 = (int)s0;
  return true;
}

// From the stencil sums L (NF fields) to the result: phase, exact FP64 add-back
// of the singular part (and its Hessian), Maxwell assembly (eq. 4.1).
template <typename T, int NF>
__device__ __forceinline__ void finish3d(const GArgs& A, double x1, double x2, double x3, const Stencil3<T>& s,
                                         const double2 L[NF], double2* res, uint8_t& fl) {
  constexpr int NO = (NF == 1) ? 1 : 6;
  if (A.smooth) {
    // the smooth part L_N(t) of Algorithm 3.1 step 2d (near branch only)
#pragma unroll
    for (int o = 0; o < NO; ++o) res[o] = L[o < NF ? o : 0];
    return;
  }
  const double t1 = s.t1, t2 = s.t2, n1 = s.n1, n2 = s.n2;
  const bool is_near = s.near;
  double ps, pc;
  sincos(A.a1 * x1 + A.a2 * x2, &ps, &pc);
  const double2 phase = mk(pc, ps);
  double2 G[NF];
#pragma unroll
  for (int f = 0; f < NF; ++f) G[f] = cmul(phase, L[f]);
  if (!is_near && NF == kMxF) {
    // d/dx3 of e^{i beta |x3|} carries sgn(x3): fields 13 and 23
    if (x3 < 0) {
      G[4] = cscale(G[4], -1.0);
      G[5] = cscale(G[5], -1.0);
    }
  }
  if (is_near) {
    // the square root only inside the support of the singular part
    const double r2 = t1 * t1 + t2 * t2 + x3 * x3;
    if (r2 <= A.rmin * A.rmin || r2 == 0.0) {
      fl |= 1;
#pragma unroll
      for (int f = 0; f < NF; ++f) G[f] = nan2();
    } else if (r2 < 4.0 * A.eps * A.eps) {
      const double r = sqrt(r2);
      // psi = e^{ikr} Y(r) / (4 pi r): the removed singular part F, times e^{i alpha.x'}
      double sn, cn;
      sincos(A.k * r, &sn, &cn);
      const double2 g = cscale(mk(cn, sn), 1.0 / (4.0 * kPi * r));
      double ls, lc;
      sincospi(2.0 * (A.a1 * n1 + A.a2 * n2), &ls, &lc);
      const double2 lat = mk(lc, ls);
      const double Y = cut_Y(r, A.eps);
      G[0] = cadd(G[0], cmul(lat, cscale(g, Y)));
      if (NF == kMxF) {
        // psi', psi'' (radial); d_p d_q psi = psi'' t_p t_q / r^2 + psi' (delta_pq / r - t_p t_q / r^3)
        const double Y1 = cut_Y1(r, A.eps), Y2 = cut_Y2(r, A.eps);
        const double2 ikr = mk(-1.0 / r, A.k);  // ik - 1/r
        const double2 g1 = cmul(g, ikr);
        const double2 g2 = cmul(g, cadd(cmul(ikr, ikr), mk(1.0 / (r * r), 0.0)));
        const double2 d1 = cadd(cscale(g1, Y), cscale(g, Y1));
        const double2 d2 = cadd(cadd(cscale(g2, Y), cscale(g1, 2.0 * Y1)), cscale(g, Y2));
        const double t[3] = {t1, t2, x3};
        const int P[5] = {0, 1, 0, 0, 1}, Qp[5] = {0, 1, 1, 2, 2};
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          const double tp = t[P[f]], tq = t[Qp[f]];
          const double a = tp * tq / (r * r);
          const double bcoef = ((P[f] == Qp[f]) ? 1.0 / r : 0.0) - tp * tq / (r * r * r);
          G[f + 1] = cadd(G[f + 1], cmul(lat, cadd(cscale(d2, a), cscale(d1, bcoef))));
        }
      }
    }
  }
  if (NF == 1) {
    res[0] = G[0];
  } else {
    // GG_pq = delta_pq G_d + k^-2 d_p d_q G_d  (eq. 4.1); fields 11 22 12 13 23, and GG_33 from
    // the trace: tr GG = 3 G_d + k^-2 Laplacian G_d = 2 G_d (the Helmholtz equation, off the lattice)
    const double ik2 = 1.0 / (A.k * A.k);
    res[0] = cadd(G[0], cscale(G[1], ik2));
    res[1] = cadd(G[0], cscale(G[2], ik2));
    res[2] = csub(cscale(G[0], 2.0), cadd(res[0], res[1]));
#pragma unroll
    for (int f = 3; f < 6; ++f) res[f] = cscale(G[f], ik2);
  }
}

// One target of Algorithm 3.1 / 4.1 step 2 (G_d, or the six Maxwell entries).
// `fetch` performs the 64-point stencil sum of the near grid or the far slab.
template <typename T, int NF, typename Fetch>
__device__ __forceinline__ void eval3d_target(const GArgs& A, double x1, double x2, double x3, const Fetch& fetch,
                                              double2* res, uint8_t& fl) {
  constexpr int NO = (NF == 1) ? 1 : 6;
  fl = 0;
  if (!(isfinite(x1) && isfinite(x2) && isfinite(x3))) {
    fl = 8;
#pragma unroll
    for (int o = 0; o < NO; ++o) res[o] = nan2();
    return;
  }
  double n1, n2;
  const double t1 = reduce_cell(x1, n1), t2 = reduce_cell(x2, n2);
  T w1[4], w2[4], w3[4];
  const double u1 = t1 * A.ih1, q1 = floor(u1);
  lag4<T>((T)(u1 - q1), w1);
  const double u2 = t2 * A.ih2, q2 = floor(u2);
  lag4<T>((T)(u2 - q2), w2);
  double2 L[NF];
  const bool is_near = fabs(x3) <= A.c;
  if (is_near) {
    const double u = x3 * A.ih3, q = floor(u);
    lag4<T>((T)(u - q), w3);
    fetch(true, (int)q1, (int)q2, (int)q, w1, w2, w3, L);
  } else {
    fl |= 2;
    if (A.smooth) {
#pragma unroll
      for (int o = 0; o < NO; ++o) res[o] = nan2();
      return;
    }
    const double v = (fabs(x3) - (A.c - A.hf)) * A.ihf;
    double s0 = floor(v);
    if (s0 > A.S - 3) {
      fl |= 4;
#pragma unroll
      for (int o = 0; o < NO; ++o) res[o] = nan2();
      return;
    }
    s0 = fmax(s0, 1.0);
    lag4<T>((T)(v - s0), w3);
    fetch(false, (int)q1, (int)q2, (int)s0, w1, w2, w3, L);
  }
  if (A.smooth) {
    // the smooth part L_N(t) of Algorithm 3.1 step 2d (near branch only)
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
  if (!is_near && NF == kMxF) {
    // d/dx3 of e^{i beta |x3|} carries sgn(x3): fields 13 and 23
    if (x3 < 0) {
      G[4] = cscale(G[4], -1.0);
      G[5] = cscale(G[5], -1.0);
    }
  }
  if (is_near) {
    // the square root only inside the support of the singular part
    const double r2 = t1 * t1 + t2 * t2 + x3 * x3;
    if (r2 <= A.rmin * A.rmin || r2 == 0.0) {
      fl |= 1;
#pragma unroll
      for (int f = 0; f < NF; ++f) G[f] = nan2();
    } else if (r2 < 4.0 * A.eps * A.eps) {
      const double r = sqrt(r2);
      // psi = e^{ikr} Y(r) / (4 pi r): the removed singular part F, times e^{i alpha.x'}
      double sn, cn;
      sincos(A.k * r, &sn, &cn);
      const double2 g = cscale(mk(cn, sn), 1.0 / (4.0 * kPi * r));
      double ls, lc;
      sincospi(2.0 * (A.a1 * n1 + A.a2 * n2), &ls, &lc);
      const double2 lat = mk(lc, ls);
      const double Y = cut_Y(r, A.eps);
      G[0] = cadd(G[0], cmul(lat, cscale(g, Y)));
      if (NF == kMxF) {
        // psi', psi'' (radial); d_p d_q psi = psi'' t_p t_q / r^2 + psi' (delta_pq / r - t_p t_q / r^3)
        const double Y1 = cut_Y1(r, A.eps), Y2 = cut_Y2(r, A.eps);
        const double2 ikr = mk(-1.0 / r, A.k);  // ik - 1/r
        const double2 g1 = cmul(g, ikr);
        const double2 g2 = cmul(g, cadd(cmul(ikr, ikr), mk(1.0 / (r * r), 0.0)));
        const double2 d1 = cadd(cscale(g1, Y), cscale(g, Y1));
        const double2 d2 = cadd(cadd(cscale(g2, Y), cscale(g1, 2.0 * Y1)), cscale(g, Y2));
        const double t[3] = {t1, t2, x3};
        const int P[5] = {0, 1, 0, 0, 1}, Qp[5] = {0, 1, 1, 2, 2};
#pragma unroll
        for (int f = 0; f < 5; ++f) {
          const double tp = t[P[f]], tq = t[Qp[f]];
          const double a = tp * tq / (r * r);
          const double bcoef = ((P[f] == Qp[f]) ? 1.0 / r : 0.0) - tp * tq / (r * r * r);
          G[f + 1] = cadd(G[f + 1], cmul(lat, cadd(cscale(d2, a), cscale(d1, bcoef))));
        }
      }
    }
  }
  if (NF == 1) {
    res[0] = G[0];
  } else {
    // GG_pq = delta_pq G_d + k^-2 d_p d_q G_d  (eq. 4.1); fields 11 22 12 13 23, and GG_33 from
    // the trace: tr GG = 3 G_d + k^-2 Laplacian G_d = 2 G_d (the Helmholtz equation, off the lattice)
    const double ik2 = 1.0 / (A.k * A.k);
    res[0] = cadd(G[0], cscale(G[1], ik2));
    res[1] = cadd(G[0], cscale(G[2], ik2));
    res[2] = csub(cscale(G[0], 2.0), cadd(res[0], res[1]));
#pragma unroll
    for (int f = 3; f < 6; ++f) res[f] = cscale(G[f], ik2);
  }
}

// 3D, unsorted targets: one thread per target, stencil read from global memory.
template <typename T, int NF>
__global__ __launch_bounds__(256) void k_gather3d(GArgs A, const cplx<T>* __restrict__ grid,
                                                  const cplx<T>* __restrict__ far, const double* __restrict__ x,
                                                  long T_, cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T_) return;
  constexpr int NO = (NF == 1) ? 1 : 6;
  const GlobalFetch<T, NF> gf{grid, far, A.fs, A.ffs, A.M1, A.M2, A.M3};
  double2 res[NO];
  uint8_t fl;
  eval3d_target<T, NF>(A, x[3 * i], x[3 * i + 1], x[3 * i + 2], gf, res, fl);
#pragma unroll
  for (int o = 0; o < NO; ++o) store_out<T>(out, i * NO + o, res[o]);
  if (flags) flags[i] = fl;
}

// ---------------------------------------------------------------------------
// Tiled gather over targets sorted by grid tile.  Tile key (see tile_key):
// near  (b3 nt2 + b2) nt1 + b1,  far  nnear + (b3 nt2 + b2) nt1 + b1,  last = invalid.
// A tile covers 2^tb nodes per axis; the stencils of its targets lie in the
// (2^tb + 3)^3 footprint starting one node before the tile.
// ---------------------------------------------------------------------------
// A target in tile order: coordinates and caller index in one aligned 32-byte record.
struct alignas(32) TRec {
  double x, y, z;
  uint32_t i, pad;
};

struct TileArgs {
  int tb1, tb2, tb3;       // tile edge = 1 << tb
  int nt1, nt2, nt3n;      // tiles along x1, x2, near x3
  int nnear, nkeys;
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

// Stencil sum from the LDS-staged footprint of one tile (compile-time footprint
// F1 x F2 x F3 so every LDS address is a base plus an immediate offset).  A
// target whose stencil does not lie in the footprint (a rounding disagreement
// with the key pass) is not evaluated here but appended to the overflow list.
template <typename T, int NF, int F1, int F2, int F3>
struct LdsFetch {
  const cplx<T>* lds;      // [NF][F3][F2][F1]
  int o1, o2, o3;
  bool near_tile;
  int M1, M2, M3;
  mutable bool miss;
  __device__ void operator()(bool near, int p1, int p2, int p3, const T w1[4], const T w2[4], const T w3[4],
                             double2 L[NF]) const {
    const int l1 = (p1 - 1 - o1) & (M1 - 1), l2 = (p2 - 1 - o2) & (M2 - 1);
    const int l3 = near ? ((p3 - 1 - o3) & (M3 - 1)) : (p3 - 1 - o3);
    if (near != near_tile || l1 > F1 - 4 || l2 > F2 - 4 || l3 < 0 || l3 > F3 - 4) {
      miss = true;
      return;
    }
    constexpr int FSZ = F1 * F2 * F3;
    const cplx<T>* base = lds + (l3 * F2 + l2) * F1 + l1;
#pragma unroll
    for (int f = 0; f < NF; ++f) L[f] = lds_sum<T, F1, F2>(base + f * FSZ, w1, w2, w3);
  }
};

template <typename T, int NF, int TB1, int TB2, int TB3, int BS>
__global__ __launch_bounds__(BS) void k_gather3d_tiled(GArgs A, TileArgs B, const cplx<T>* __restrict__ grid,
                                                        const cplx<T>* __restrict__ far,
                                                        const TRec* __restrict__ rec,
                                                        const uint32_t* __restrict__ hist,
                                                        const uint32_t* __restrict__ offs,
                                                        cplx<T>* __restrict__ out, uint8_t* __restrict__ flags,
                                                        uint32_t* __restrict__ ovf, uint32_t* __restrict__ novf) {
  constexpr int F1 = (1 << TB1) + 3, F2 = (1 << TB2) + 3, F3 = (1 << TB3) + 3, FSZ = F1 * F2 * F3;
  __shared__ cplx<T> lds[NF * FSZ];
  constexpr int NO = (NF == 1) ? 1 : 6;
  // far tiles (more targets each, keys >= nnear) first, then near tiles; blocks go
  // round-robin over the XCDs so every XCD gets the same mix
  const int key = B.nkeys - 1 - (int)blockIdx.x;
  const uint32_t cnt = hist[key];
  if (cnt == 0) return;
  const long start = offs[key];
  if (key >= B.nkeys - 1) {
    // non-finite targets and targets beyond the far slab: NaN and their flags
    const GlobalFetch<T, NF> gf{grid, far, A.fs, A.ffs, A.M1, A.M2, A.M3};
    for (long j = start + threadIdx.x; j < start + (long)cnt; j += blockDim.x) {
      const TRec r = rec[j];
      const long i = r.i;
      double2 res[NO];
      uint8_t fl;
      eval3d_target<T, NF>(A, r.x, r.y, r.z, gf, res, fl);
#pragma unroll
      for (int o = 0; o < NO; ++o) store_out<T>(out, i * NO + o, res[o]);
      if (flags) flags[i] = fl;
    }
    return;
  }
  LdsFetch<T, NF, F1, F2, F3> lf;
  lf.lds = lds;
  lf.M1 = A.M1;
  lf.M2 = A.M2;
  lf.M3 = A.M3;
  const bool near = key < B.nnear;
  const int kk = near ? key : key - B.nnear;
  const int b1 = kk % B.nt1, b2 = (kk / B.nt1) % B.nt2, b3 = kk / (B.nt1 * B.nt2);
  lf.near_tile = near;
  lf.o1 = (b1 << TB1) - 1;
  lf.o2 = (b2 << TB2) - 1;
  lf.o3 = (b3 << TB3) - 1;
  for (int idx = threadIdx.x; idx < NF * FSZ; idx += blockDim.x) {
    const int f = idx / FSZ, r = idx - f * FSZ;
    const int z = r / (F1 * F2), y = (r / F1) % F2, xx = r % F1;
    const int g1 = (lf.o1 + xx) & (A.M1 - 1), g2 = (lf.o2 + y) & (A.M2 - 1);
    cplx<T> v;
    if (near) {
      const int g3 = (lf.o3 + z) & (A.M3 - 1);
      v = grid[f * A.fs + ((long)g3 * A.M2 + g2) * A.M1 + g1];
    } else {
      const int g3 = min(max(lf.o3 + z, 0), A.S - 1);
      v = far[f * A.ffs + ((long)g3 * A.M2 + g2) * A.M1 + g1];
    }
    lds[idx] = v;
  }
  __syncthreads();
  // the next record is loaded before the current one is evaluated
  const long end = start + (long)cnt;
  long j = start + threadIdx.x;
  TRec r{};
  if (j < end) r = rec[j];
  for (; j < end; j += BS) {
    TRec rn = r;
    if (j + BS < end) rn = rec[j + BS];
    double2 res[NO];
    uint8_t fl;
    lf.miss = false;
    eval3d_target<T, NF>(A, r.x, r.y, r.z, lf, res, fl);
    if (lf.miss) {
      ovf[atomicAdd(novf, 1u)] = (uint32_t)j;
    } else {
      const long i = r.i;
#pragma unroll
      for (int o = 0; o < NO; ++o) store_out<T>(out, i * NO + o, res[o]);
      if (flags) flags[i] = fl;
    }
    r = rn;
  }
}

// Maxwell tensor over targets sorted by tile, one field at a time: the tile's
// footprint of field f is staged in LDS, every target of the tile takes its
// stencil sum of field f, then the next field replaces it.  Used when the tiles
// hold few targets (fewer than about two blocks' worth), so a footprint of all
// six fields would not fit LDS at a useful tile size.  Up to 256 targets per
// pass; a tile with more runs several passes, staging again.
template <typename T, int TB1, int TB2, int TB3>
__global__ __launch_bounds__(256) void k_gather3d_fields(GArgs A, TileArgs B, const cplx<T>* __restrict__ grid,
                                                         const cplx<T>* __restrict__ far,
                                                         const TRec* __restrict__ rec,
                                                         const uint32_t* __restrict__ hist,
                                                         const uint32_t* __restrict__ offs,
                                                         cplx<T>* __restrict__ out, uint8_t* __restrict__ flags,
                                                         uint32_t* __restrict__ ovf, uint32_t* __restrict__ novf) {
  constexpr int F1 = (1 << TB1) + 3, F2 = (1 << TB2) + 3, F3 = (1 << TB3) + 3, FSZ = F1 * F2 * F3;
  constexpr int NF = kMxF, NO = 6;
  __shared__ cplx<T> lds[FSZ];
  const int key = B.nkeys - 1 - (int)blockIdx.x;
  const uint32_t cnt = hist[key];
  if (cnt == 0) return;
  const long start = offs[key];
  if (key >= B.nkeys - 1) {
    const GlobalFetch<T, NF> gf{grid, far, A.fs, A.ffs, A.M1, A.M2, A.M3};
    for (long j = start + threadIdx.x; j < start + (long)cnt; j += blockDim.x) {
      const TRec r = rec[j];
      double2 res[NO];
      uint8_t fl;
      eval3d_target<T, NF>(A, r.x, r.y, r.z, gf, res, fl);
#pragma unroll
      for (int o = 0; o < NO; ++o) store_out<T>(out, (long)r.i * NO + o, res[o]);
      if (flags) flags[r.i] = fl;
    }
    return;
  }
  const bool near = key < B.nnear;
  const int kk = near ? key : key - B.nnear;
  const int b1 = kk % B.nt1, b2 = (kk / B.nt1) % B.nt2, b3 = kk / (B.nt1 * B.nt2);
  const int o1 = (b1 << TB1) - 1, o2 = (b2 << TB2) - 1, o3 = (b3 << TB3) - 1;
  for (long c0 = 0; c0 < (long)cnt; c0 += blockDim.x) {
    const long j = start + c0 + threadIdx.x;
    const bool valid = c0 + (long)threadIdx.x < (long)cnt;
    TRec r{};
    Stencil3<T> st;
    double2 res[NO];
    uint8_t fl = 0;
    bool go = false, miss = false;
    int l1 = 0, l2 = 0, l3 = 0;
    if (valid) {
      r = rec[j];
      go = stencil3d<T, NO>(A, r.x, r.y, r.z, st, res, fl);
      if (go) {
        l1 = (st.p1 - 1 - o1) & (A.M1 - 1);
        l2 = (st.p2 - 1 - o2) & (A.M2 - 1);
        l3 = st.near ? ((st.p3 - 1 - o3) & (A.M3 - 1)) : (st.p3 - 1 - o3);
        miss = st.near != near || l1 > F1 - 4 || l2 > F2 - 4 || l3 < 0 || l3 > F3 - 4;
      }
    }
    double2 L[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      __syncthreads();   // the previous field's sums are done
      for (int idx = threadIdx.x; idx < FSZ; idx += blockDim.x) {
        const int z = idx / (F1 * F2), y = (idx / F1) % F2, xx = idx % F1;
        const int g1 = (o1 + xx) & (A.M1 - 1), g2 = (o2 + y) & (A.M2 - 1);
        cplx<T> v;
        if (near) {
          const int g3 = (o3 + z) & (A.M3 - 1);
          v = grid[f * A.fs + ((long)g3 * A.M2 + g2) * A.M1 + g1];
        } else {
          const int g3 = min(max(o3 + z, 0), A.S - 1);
          v = far[f * A.ffs + ((long)g3 * A.M2 + g2) * A.M1 + g1];
        }
        lds[idx] = v;
      }
      __syncthreads();
      if (go && !miss) L[f] = lds_sum<T, F1, F2>(lds + (l3 * F2 + l2) * F1 + l1, st.w1, st.w2, st.w3);
    }
    if (!valid) continue;
    if (go && miss) {
      ovf[atomicAdd(novf, 1u)] = (uint32_t)j;
      continue;
    }
    if (go) finish3d<T, NF>(A, r.x, r.y, r.z, st, L, res, fl);
#pragma unroll
    for (int o = 0; o < NO; ++o) store_out<T>(out, (long)r.i * NO + o, res[o]);
    if (flags) flags[r.i] = fl;
  }
}

// Targets the tiled kernel handed over (stencil outside its tile footprint):
// evaluated from global memory.  The count is read on the device.
template <typename T, int NF>
__global__ __launch_bounds__(256) void k_gather3d_overflow(GArgs A, const cplx<T>* __restrict__ grid,
                                                           const cplx<T>* __restrict__ far,
                                                           const TRec* __restrict__ rec,
                                                           const uint32_t* __restrict__ ovf,
                                                           const uint32_t* __restrict__ novf,
                                                           cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  constexpr int NO = (NF == 1) ? 1 : 6;
  const GlobalFetch<T, NF> gf{grid, far, A.fs, A.ffs, A.M1, A.M2, A.M3};
  const long n = *novf;
  for (long q = (long)blockIdx.x * blockDim.x + threadIdx.x; q < n; q += (long)gridDim.x * blockDim.x) {
    const TRec r = rec[ovf[q]];
    const long i = r.i;
    double2 res[NO];
    uint8_t fl;
    eval3d_target<T, NF>(A, r.x, r.y, r.z, gf, res, fl);
#pragma unroll
    for (int o = 0; o < NO; ++o) store_out<T>(out, i * NO + o, res[o]);
    if (flags) flags[i] = fl;
  }
}

// 2D: G (Algorithm 2.1).
// 4 x 4 stencil sum of a 2D grid: rows[b] is the first element of stencil row b, i0 the
// first x1 node (periodic in x1).
template <typename T>
__device__ __forceinline__ double2 stencil2d_scalar(const cplx<T>* __restrict__ g, const long rows[4], int i0,
                                                    int M1, const T w1[4], const T w2[4]) {
  Acc<T> acc;
#pragma unroll
  for (int b = 0; b < 4; ++b)
#pragma unroll
    for (int a = 0; a < 4; ++a) acc.add(w2[b] * w1[a], g[rows[b] + ((i0 + a) & (M1 - 1))]);
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
      rs[b] = row4v(g[rows[b] + i0], g[rows[b] + ((i0 + 1) & (M1 - 1))], g[rows[b] + ((i0 + 2) & (M1 - 1))],
                    g[rows[b] + ((i0 + 3) & (M1 - 1))], w1);
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
      const cplx<T>* q = g + (rows[b] + ((i0 + a) & (M1 - 1))) * NF;
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
    T w1[4], w2[4];
    const double u = t * A.ih1, p = floor(u);
    lag4<T>((T)(u - p), w1);
    const int i0 = ((int)p - 1) & (A.M1 - 1);
    double ps, pc;
    sincos(A.a1 * x1, &ps, &pc);
    const double2 phase = mk(pc, ps);
    const bool is_near = fabs(x2) <= A.c;
    long rows[4];
    const cplx<T>* g = grid;
    bool bad = false;
    if (is_near) {
      const double u2 = x2 * A.ih2, p2 = floor(u2);
      lag4<T>((T)(u2 - p2), w2);
#pragma unroll
      for (int b = 0; b < 4; ++b) rows[b] = (long)(((int)p2 - 1 + b) & (A.M2 - 1)) * A.M1;
    } else {
      fl |= 2;
      g = far;
      const double v = (fabs(x2) - (A.c - A.hf)) * A.ihf;
      double s0 = floor(v);
      if (s0 > A.S - 3) {
        bad = true;
        fl |= 4;
      } else {
        s0 = fmax(s0, 1.0);
        lag4<T>((T)(v - s0), w2);
#pragma unroll
        for (int b = 0; b < 4; ++b) rows[b] = ((long)s0 - 1 + b) * A.M1;
      }
    }
    if (bad) {
      res = nan2();
    } else {
      double2 Lt;
      if constexpr (sizeof(T) == 4) {
        if (A.quad) Lt = stencil2d_quad(g, rows, i0, w1, w2);
        else Lt = stencil2d<T>(g, rows, i0, A.M1, w1, w2);
      } else {
        Lt = stencil2d<T>(g, rows, i0, A.M1, w1, w2);
      }
      if (is_near) {
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
      }
      res = cmul(phase, Lt);
    }
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
// point.  The complex128 path computes in FP64, the complex64 path in FP32 (the correction is a
// small part of a result kept to single precision; the phase stays FP64).  Each block takes
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
    T w1[4], w2[4];
    lag4<T>((T)(u - p), w1);
    lag4<T>((T)(u2 - p2), w2);
    // NF = 1: f Y of the 2D G; NF = 2: the gradient's h1, h2; NF = 3: h_11, h_12, h_22
    cplx<T> acc[NF], at[NF];
#pragma unroll
    for (int f = 0; f < NF; ++f) acc[f] = cv<T>(0, 0);
    for (int b = 0; b < 4; ++b) {
      const T zn = (T)((p2 - 1.0 + b) * A.h2);
      cplx<T> row[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) row[f] = cv<T>(0, 0);
      for (int a = 0; a < 4; ++a) {
        const T tn = (T)((p - 1.0 + a) * A.h1);
        cplx<T> v[NF];
        if constexpr (NF == 1) v[0] = fy_removed<T>(A, tn, zn);
        else if constexpr (NF == 2) hgrad_at<T>(A, tn, zn, v[0], v[1]);
        else hhess_at<T>(A, tn, zn, v);
#pragma unroll
        for (int f = 0; f < NF; ++f) row[f] = cv<T>(fma(w1[a], v[f].x, row[f].x), fma(w1[a], v[f].y, row[f].y));
      }
#pragma unroll
      for (int f = 0; f < NF; ++f) acc[f] = cv<T>(fma(w2[b], row[f].x, acc[f].x), fma(w2[b], row[f].y, acc[f].y));
    }
    if constexpr (NF == 1) at[0] = fy_removed<T>(A, (T)t, (T)x2);
    else if constexpr (NF == 2) hgrad_at<T>(A, (T)t, (T)x2, at[0], at[1]);
    else hhess_at<T>(A, (T)t, (T)x2, at);
    double ps, pc;
    sincos(A.a1 * x1, &ps, &pc);
#pragma unroll
    for (int f = 0; f < NF; ++f) {
      const double2 corr = cmul(mk(pc, ps), mk((double)(acc[f].x - at[f].x), (double)(acc[f].y - at[f].y)));
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
// e^{i alpha x1}; beyond c the differentiated far slab, the x2 field times sgn(x2).
// grid and far hold the two fields interleaved per node.  out[2i] = dG/dx1, out[2i+1] = dG/dx2.
// Returns whether the target lies in the cut-off ring (when the plan marks them).
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
    T w1[4], w2[4];
    const double u = t * A.ih1, p = floor(u);
    lag4<T>((T)(u - p), w1);
    const int i0 = ((int)p - 1) & (A.M1 - 1);
    double ps, pc;
    sincos(A.a1 * x1, &ps, &pc);
    const double2 phase = mk(pc, ps);
    const bool is_near = fabs(x2) <= A.c;
    long rows[4];
    const cplx<T>* g = grid;
    bool bad = false;
    if (is_near) {
      const double u2 = x2 * A.ih2, p2 = floor(u2);
      lag4<T>((T)(u2 - p2), w2);
#pragma unroll
      for (int b = 0; b < 4; ++b) rows[b] = (long)(((int)p2 - 1 + b) & (A.M2 - 1)) * A.M1;
    } else {
      fl |= 2;
      g = far;
      const double v = (fabs(x2) - (A.c - A.hf)) * A.ihf;
      double s0 = floor(v);
      if (s0 > A.S - 3) {
        bad = true;
        fl |= 4;
      } else {
        s0 = fmax(s0, 1.0);
        lag4<T>((T)(v - s0), w2);
#pragma unroll
        for (int b = 0; b < 4; ++b) rows[b] = ((long)s0 - 1 + b) * A.M1;
      }
    }
    if (bad) {
      d1 = d2 = nan2();
    } else {
      double2 L[2];
      stencil2d_fields<T, 2>(g, rows, i0, A.M1, w1, w2, L);
      double2 L1 = L[0], L2 = L[1];
      if (is_near) {
        const double r2 = t * t + x2 * x2;
        if (r2 <= A.rmin * A.rmin || r2 == 0.0) {
          fl |= 1;
          L1 = L2 = nan2();
        } else {
          if (r2 < 4.0 * A.eps * A.eps) {
            double2 h1, h2;
            hgrad_at(A, t, x2, h1, h2);
            L1 = cadd(L1, h1);
            L2 = cadd(L2, h2);
          }
          if (A.ring_mask) {
            const double r = sqrt(r2);
            in_ring = r > A.ring_lo && r < A.ring_hi;
          }
        }
      } else if (x2 < 0.0) {
        L2 = cscale(L2, -1.0);
      }
      d1 = cmul(phase, L1);
      d2 = cmul(phase, L2);
    }
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
// slab, the 12 field times sgn(x2).  grid and far hold the three fields interleaved per node.
// out[3i + p] = d_p d_q G_k1 - d_p d_q G_k2, pq = 11, 12, 22.
template <typename T>
__device__ __forceinline__ bool gather2d_hess_one(const GArgs& A, const cplx<T>* __restrict__ grid,
                                                  const cplx<T>* __restrict__ far, const double* __restrict__ x,
                                                  long i, cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  const double x1 = x[2 * i], x2 = x[2 * i + 1];
  uint8_t fl = 0;
  bool in_ring = false;
  double2 d[3];
  if (!(isfinite(x1) && isfinite(x2))) {
    fl = 8;
    d[0] = d[1] = d[2] = nan2();
  } else {
    double n1;
    const double t = reduce_cell(x1, n1);
    T w1[4], w2[4];
    const double u = t * A.ih1, p = floor(u);
    lag4<T>((T)(u - p), w1);
    const int i0 = ((int)p - 1) & (A.M1 - 1);
    double ps, pc;
    sincos(A.a1 * x1, &ps, &pc);
    const double2 phase = mk(pc, ps);
    const bool is_near = fabs(x2) <= A.c;
    long rows[4];
    const cplx<T>* g = grid;
    bool bad = false;
    if (is_near) {
      const double u2 = x2 * A.ih2, p2 = floor(u2);
      lag4<T>((T)(u2 - p2), w2);
#pragma unroll
      for (int b = 0; b < 4; ++b) rows[b] = (long)(((int)p2 - 1 + b) & (A.M2 - 1)) * A.M1;
    } else {
      fl |= 2;
      g = far;
      const double v = (fabs(x2) - (A.c - A.hf)) * A.ihf;
      double s0 = floor(v);
      if (s0 > A.S - 3) {
        bad = true;
        fl |= 4;
      } else {
        s0 = fmax(s0, 1.0);
        lag4<T>((T)(v - s0), w2);
#pragma unroll
        for (int b = 0; b < 4; ++b) rows[b] = ((long)s0 - 1 + b) * A.M1;
      }
    }
    if (bad) {
      d[0] = d[1] = d[2] = nan2();
    } else {
      double2 L[3];
      stencil2d_fields<T, 3>(g, rows, i0, A.M1, w1, w2, L);
      if (is_near) {
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
      } else if (x2 < 0.0) {
        L[1] = cscale(L[1], -1.0);
      }
#pragma unroll
      for (int f = 0; f < 3; ++f) d[f] = cmul(phase, L[f]);
    }
  }
#pragma unroll
  for (int f = 0; f < 3; ++f) store_out<T>(out, 3 * i + f, d[f]);
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
  double c, ih1, ih2, ih3, hf, ihf;
  int M1, M2, M3, S;
  TileArgs t;
};

__device__ __forceinline__ uint32_t tile_key(const BinArgs& B, double x1, double x2, double x3) {
  if (!(isfinite(x1) && isfinite(x2) && isfinite(x3))) return B.t.nkeys - 1;
  double n;
  const double t1 = reduce_cell(x1, n), t2 = reduce_cell(x2, n);
  const int b1 = (((int)floor(t1 * B.ih1)) & (B.M1 - 1)) >> B.t.tb1;
  const int b2 = (((int)floor(t2 * B.ih2)) & (B.M2 - 1)) >> B.t.tb2;
  if (fabs(x3) <= B.c) {
    const int b3 = (((int)floor(x3 * B.ih3)) & (B.M3 - 1)) >> B.t.tb3;
    return (uint32_t)((b3 * B.t.nt2 + b2) * B.t.nt1 + b1);
  }
  const double s0 = floor((fabs(x3) - (B.c - B.hf)) * B.ihf);
  if (s0 > B.S - 3) return B.t.nkeys - 1;
  const int b3 = ((int)fmax(s0, 1.0)) >> B.t.tb3;
  return (uint32_t)(B.t.nnear + (b3 * B.t.nt2 + b2) * B.t.nt1 + b1);
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

// exclusive scan of hist[0..n) into offs[0..n) with one block of 1024 threads
__global__ __launch_bounds__(1024) void k_bin_scan(const uint32_t* __restrict__ hist, uint32_t* __restrict__ offs,
                                                   int n) {
  __shared__ uint32_t part[1024];
  const int t = threadIdx.x, per = (n + 1023) / 1024;
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
constexpr int kBinUnroll = 4;
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
  q[v] = in[row * M1 + ((i1 + a) & (M1 - 1))];
}

enum GatherMode { kGatherAll = 0, kBinOnly = 1, kGatherBinned = 2 };

template <typename T>
hipError_t gather_impl(Plan& P, const double* x, int64_t T_, void* out, uint8_t* flags, int smooth = 0,
                       int mode = kGatherAll, hipStream_t bin_stream = nullptr) {
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
  A.hf = P.p.far_h;
  A.ihf = 1.0 / A.hf;
  A.S = P.S;
  A.fs = (long)P.ncell;
  A.ffs = (long)P.nfar;
  A.smooth = smooth;
  A.sing_order = P.p.sing_order;
  A.quad = P.dim == 2 && P.nf == 1 && P.gridI != nullptr;
  A.ring_mask = nullptr;
  // the ring zone r_lo < r < r_hi: r_hi = 2 eps + 2 sqrt(2) h, beyond which every stencil node has
  // Y = 0; r_lo = max(eps, eps/2 + 2 sqrt(2) h) keeps every node at least eps/2 from the lattice point
  const double reach = 2.0 * sqrt(2.0) * fmax(A.h1, A.h2);
  A.ring_lo = fmax(A.eps, 0.5 * A.eps + reach);
  A.ring_hi = 2.0 * A.eps + reach;
  const auto* g = static_cast<const cplx<T>*>(P.grid);
  const auto* f = static_cast<const cplx<T>*>(P.far);
  auto* o = static_cast<cplx<T>*>(out);
  const dim3 grid((unsigned)((T_ + 255) / 256));
  if (smooth) {
    KernelTimer t(P, QPGF_T_GATHER);
    hipLaunchKernelGGL((k_gather3d<T, 1>), grid, dim3(256), 0, P.stream, A, g, f, x, (long)T_, o, flags);
    return hipGetLastError();
  }
  if (P.dim == 2) {
    const auto* gi = static_cast<const cplx<T>*>(P.gridI);
    const auto* fi = static_cast<const cplx<T>*>(P.farI);
    if (P.p.ring_interp) {
      hipError_t e = ensure_ring_scratch(P, T_);
      if (e != hipSuccess) return e;
      A.ring_mask = P.ring_mask;
    }
    {
      KernelTimer t(P, QPGF_T_GATHER);   // the gather alone; the ring pass has its own timer
      if (P.nf == 2)
        hipLaunchKernelGGL(k_gather2d_grad<T>, grid, dim3(256), 0, P.stream, A, gi, fi, x, (long)T_, o, flags);
      else if (P.nf == 3)
        hipLaunchKernelGGL(k_gather2d_hess<T>, grid, dim3(256), 0, P.stream, A, gi, fi, x, (long)T_, o, flags);
      else
        hipLaunchKernelGGL(k_gather2d<T>, grid, dim3(256), 0, P.stream, A, A.quad ? gi : g, A.quad ? fi : f, x,
                           (long)T_, o, flags);
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
  if (P.bin_min_targets < 0 || T_ < P.bin_min_targets) {
    KernelTimer t(P, QPGF_T_GATHER);
    if (P.nf == kMxF)
      hipLaunchKernelGGL((k_gather3d<T, kMxF>), grid, dim3(256), 0, P.stream, A, g, f, x, (long)T_, o, flags);
    else
      hipLaunchKernelGGL((k_gather3d<T, 1>), grid, dim3(256), 0, P.stream, A, g, f, x, (long)T_, o, flags);
    return hipGetLastError();
  }
  BinArgs B;
  B.c = A.c;
  B.ih1 = A.ih1;
  B.ih2 = A.ih2;
  B.ih3 = A.ih3;
  B.hf = A.hf;
  B.ihf = A.ihf;
  B.M1 = P.M1;
  B.M2 = P.M2;
  B.M3 = P.M3;
  B.S = P.S;
  // Tile edges.  One field: 16 x 16 x 8 nodes (several 256-thread blocks per
  // CU, so one block's staging overlaps the others' interpolation), or, when
  // that leaves fewer than kMinPerTile targets per tile on average (fine grids),
  // 32 x 32 x 8 (complex64, 108 KiB, 1024 threads) or 32 x 16 x 8 (complex128,
  // 117 KiB, 512 threads) so the staging is spread over more targets.  Seven
  // Maxwell fields: 8 x 8 x 4 (complex64) or 8 x 4 x 4 (complex128) so the
  // staged footprint fits in 64 KiB.  Must match the instantiations of
  // k_gather3d_tiled below.
  TileArgs& Tl = B.t;
  auto set_tiles = [&](int a, int b, int c) {
    Tl.tb1 = a;
    Tl.tb2 = b;
    Tl.tb3 = c;
    Tl.nt1 = std::max(1, P.M1 >> Tl.tb1);
    Tl.nt2 = std::max(1, P.M2 >> Tl.tb2);
    Tl.nt3n = std::max(1, P.M3 >> Tl.tb3);
    Tl.nnear = Tl.nt1 * Tl.nt2 * Tl.nt3n;
    Tl.nkeys = Tl.nnear + Tl.nt1 * Tl.nt2 * ((P.S >> Tl.tb3) + 1) + 1;
  };
  bool big = false, fields = false;
  hipError_t e = hipSuccess;
  if (mode == kGatherBinned) {
    // the configuration launch_bin3d used for these targets
    if (P.bt_T != T_ || P.bt_x != x) return hipErrorInvalidValue;
    Tl.tb1 = P.bt[0];
    Tl.tb2 = P.bt[1];
    Tl.tb3 = P.bt[2];
    Tl.nt1 = P.bt[3];
    Tl.nt2 = P.bt[4];
    Tl.nt3n = P.bt[5];
    Tl.nnear = P.bt[6];
    Tl.nkeys = P.bt[7];
    big = P.bt_big;
    fields = P.bt_fields;
  } else {
    if (P.nf == kMxF) {
      // few targets per tile: 16 x 16 x 8 tiles staged one field at a time
      set_tiles(4, 4, 3);
      fields = T_ < (int64_t)kMaxPerFieldTile * Tl.nkeys;
      if (!fields) set_tiles(3, sizeof(T) == 8 ? 2 : 3, 2);
    } else {
      set_tiles(4, 4, 3);
      if (T_ < (int64_t)kMinPerTile * Tl.nkeys) {
        big = true;
        set_tiles(5, sizeof(T) == 8 ? 4 : 5, 3);
      }
    }
    e = ensure_bin_scratch(P, T_, Tl.nkeys);
    if (e != hipSuccess) return e;
    const int bt[8] = {Tl.tb1, Tl.tb2, Tl.tb3, Tl.nt1, Tl.nt2, Tl.nt3n, Tl.nnear, Tl.nkeys};
    for (int q = 0; q < 8; ++q) P.bt[q] = bt[q];
    P.bt_big = big;
    P.bt_fields = fields;
    P.bt_T = T_;
    P.bt_x = x;
  }
  TRec* rec = reinterpret_cast<TRec*>(P.bin_rec);
  const bool lds_bins = Tl.nkeys <= kBinLdsKeys;
  const long chunk = (T_ + kBinBlocks - 1) / kBinBlocks;
  const hipStream_t bs = bin_stream ? bin_stream : P.stream;
  if (mode != kGatherBinned) {
  {
    KernelTimer t(P, QPGF_T_BIN, bs);
    hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, bs, P.bin_novf, 1L);
    if (lds_bins) {
      // LDS histogram sized to the key count (small ones leave LDS to kernels running beside)
      if (Tl.nkeys <= 4096)
        hipLaunchKernelGGL(k_bin_count<4096>, dim3(kBinBlocks), dim3(1024), 0, bs, B, x, (long)T_, chunk, P.bin_cnt);
      else if (Tl.nkeys <= 16384)
        hipLaunchKernelGGL(k_bin_count<16384>, dim3(kBinBlocks), dim3(1024), 0, bs, B, x, (long)T_, chunk, P.bin_cnt);
      else
        hipLaunchKernelGGL(k_bin_count<kBinLdsKeys>, dim3(kBinBlocks), dim3(1024), 0, bs, B, x, (long)T_, chunk,
                           P.bin_cnt);
      hipLaunchKernelGGL(k_bin_colscan, dim3((Tl.nkeys + 63) / 64), dim3(64 * kColGroups), 0, bs, P.bin_cnt,
                         Tl.nkeys,
                         kBinBlocks, P.bin_hist);
    } else {
      // large key spaces: one global atomic rank per target
      hipLaunchKernelGGL(k_zero_u32, dim3((Tl.nkeys + 255) / 256), dim3(256), 0, bs, P.bin_hist,
                         (long)Tl.nkeys);
      hipLaunchKernelGGL(k_bin_key, grid, dim3(256), 0, bs, B, x, (long)T_, P.bin_hist, P.bin_keyrank);
    }
    hipLaunchKernelGGL(k_bin_scan, dim3(1), dim3(1024), 0, bs, P.bin_hist, P.bin_offs, Tl.nkeys);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    KernelTimer t(P, QPGF_T_BIN_PLACE, bs);
    if (lds_bins && Tl.nkeys <= 4096)
      hipLaunchKernelGGL(k_bin_place<4096>, dim3(kBinBlocks), dim3(1024), 0, bs, B, x, (long)T_, chunk, P.bin_cnt,
                         P.bin_offs, rec);
    else if (lds_bins && Tl.nkeys <= 16384)
      hipLaunchKernelGGL(k_bin_place<16384>, dim3(kBinBlocks), dim3(1024), 0, bs, B, x, (long)T_, chunk, P.bin_cnt,
                         P.bin_offs, rec);
    else if (lds_bins)
      hipLaunchKernelGGL(k_bin_place<kBinLdsKeys>, dim3(kBinBlocks), dim3(1024), 0, bs, B, x, (long)T_, chunk,
                         P.bin_cnt, P.bin_offs, rec);
    else
      hipLaunchKernelGGL(k_bin_scatter, grid, dim3(256), 0, bs, x, P.bin_keyrank, P.bin_offs, (long)T_, rec);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  }
  if (mode == kBinOnly) return hipSuccess;
  {
  KernelTimer t(P, QPGF_T_GATHER);
  const dim3 tg(Tl.nkeys);
#define QPGF_TILED(NF_, A1_, A2_, A3_, BS_)                                                                      \
  hipLaunchKernelGGL((k_gather3d_tiled<T, NF_, A1_, A2_, A3_, BS_>), tg, dim3(BS_), 0, P.stream, A, Tl, g, f, rec, \
                     P.bin_hist, P.bin_offs, o, flags, P.bin_ovf, P.bin_novf)
  if (fields) {
    hipLaunchKernelGGL((k_gather3d_fields<T, 4, 4, 3>), tg, dim3(256), 0, P.stream, A, Tl, g, f, rec, P.bin_hist,
                       P.bin_offs, o, flags, P.bin_ovf, P.bin_novf);
  } else if constexpr (sizeof(T) == 8) {
    if (P.nf == kMxF) QPGF_TILED(kMxF, 3, 2, 2, 256);
    else if (big) QPGF_TILED(1, 5, 4, 3, 512);
    else QPGF_TILED(1, 4, 4, 3, 256);
  } else {
    if (P.nf == kMxF) QPGF_TILED(kMxF, 3, 3, 2, 256);
    else if (big) QPGF_TILED(1, 5, 5, 3, 1024);
    else QPGF_TILED(1, 4, 4, 3, 256);
  }
#undef QPGF_TILED
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  }
  KernelTimer t(P, QPGF_T_OVERFLOW);
  if (P.nf == kMxF)
    hipLaunchKernelGGL((k_gather3d_overflow<T, kMxF>), dim3(64), dim3(256), 0, P.stream, A, g, f, rec, P.bin_ovf,
                       P.bin_novf, o, flags);
  else
    hipLaunchKernelGGL((k_gather3d_overflow<T, 1>), dim3(64), dim3(256), 0, P.stream, A, g, f, rec, P.bin_ovf,
                       P.bin_novf, o, flags);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_interleave2d(Plan& P) {
  if (P.dim != 2 || !P.gridI || !P.farI) return hipErrorInvalidValue;
  if (P.nf == 1) {
    // complex64 G: node quads of the near grid and of the far slab
    if (P.esize != 8) return hipErrorInvalidValue;
    auto quads = [&](const void* in, void* out, long n) {
      hipLaunchKernelGGL(k_quads, dim3((unsigned)((4 * n + 255) / 256)), dim3(256), 0, P.stream,
                         static_cast<const float2*>(in), static_cast<float2*>(out), n, P.M1);
    };
    quads(P.grid, P.gridI, (long)P.ncell);
    quads(P.far, P.farI, (long)P.nfar);
    return hipGetLastError();
  }
  auto go = [&](auto tag, const void* in, void* out, long n) {
    using T = decltype(tag);
    const long tot = n * P.nf;
    hipLaunchKernelGGL(k_interleave<T>, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, P.stream,
                       static_cast<const cplx<T>*>(in), static_cast<cplx<T>*>(out), n, P.nf);
  };
  if (P.esize == 16) {
    go(double(), P.grid, P.gridI, (long)P.ncell);
    go(double(), P.far, P.farI, (long)P.nfar);
  } else {
    go(float(), P.grid, P.gridI, (long)P.ncell);
    go(float(), P.far, P.farI, (long)P.nfar);
  }
  return hipGetLastError();
}

hipError_t ensure_ring_scratch(Plan& P, int64_t T_) {
  const int64_t words = (T_ + 63) / 64;
  if (words <= P.ring_words) return hipSuccess;
  if (P.ring_mask) (void)hipFree(P.ring_mask);
  P.ring_mask = nullptr;
  P.ring_words = 0;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&P.ring_mask), (size_t)words * sizeof(unsigned long long));
  if (e != hipSuccess) return e;
  P.ring_words = words;
  return hipSuccess;
}

hipError_t ensure_bin_scratch(Plan& P, int64_t T_, int nkeys) {
  if (T_ > P.bin_cap) {
    for (void* q : {(void*)P.bin_keyrank, (void*)P.bin_rec, (void*)P.bin_ovf})
      if (q) (void)hipFree(q);
    P.bin_keyrank = nullptr;
    P.bin_rec = nullptr;
    P.bin_ovf = nullptr;
    P.bin_cap = 0;
    hipError_t e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&P.bin_keyrank), (size_t)T_ * sizeof(uint2))) != hipSuccess) return e;
    if ((e = hipMalloc(&P.bin_rec, (size_t)T_ * sizeof(TRec))) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&P.bin_ovf), (size_t)T_ * sizeof(uint32_t))) != hipSuccess) return e;
    P.bin_cap = T_;
  }
  if (nkeys > P.bin_keycap) {
    for (void* q : {(void*)P.bin_hist, (void*)P.bin_offs, (void*)P.bin_cnt})
      if (q) (void)hipFree(q);
    P.bin_hist = nullptr;
    P.bin_offs = nullptr;
    P.bin_cnt = nullptr;
    P.bin_keycap = 0;
    hipError_t e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&P.bin_hist), (size_t)nkeys * sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&P.bin_offs), (size_t)nkeys * sizeof(uint32_t))) != hipSuccess) return e;
    if (!P.bin_novf && (e = hipMalloc(reinterpret_cast<void**>(&P.bin_novf), sizeof(uint32_t))) != hipSuccess) return e;
    if ((e = hipMalloc(reinterpret_cast<void**>(&P.bin_cnt), (size_t)nkeys * kBinBlocks * sizeof(uint32_t))) !=
        hipSuccess)
      return e;
    P.bin_keycap = nkeys;
  }
  return hipSuccess;
}

void gather_inst_2d(const Plan& P, double k, double a, int M1, long off, long foff, long t0, long t1, long blk0,
                    void* dst) {
  GatherInst I;
  GArgs& A = I.A;
  A.k = k;
  A.a1 = a;
  A.a2 = 0.0;
  A.c = P.p.c;
  A.c_tilde = P.p.c_tilde;
  A.eps = P.p.eps;
  A.rmin = P.p.lattice_rmin;
  A.M1 = M1;
  A.M2 = P.M2;
  A.M3 = 1;
  A.h1 = kPi / (M1 / 2);
  A.h2 = P.p.c_tilde / (P.M2 / 2);
  A.h3 = 0.0;
  A.ih1 = 1.0 / A.h1;
  A.ih2 = 1.0 / A.h2;
  A.ih3 = 0.0;
  A.hf = P.p.far_h;
  A.ihf = 1.0 / A.hf;
  A.S = P.S;
  A.fs = (long)M1 * P.M2;
  A.ffs = (long)M1 * P.S;
  A.smooth = 0;
  A.sing_order = P.p.sing_order;
  A.quad = 0;   // the batched graph keeps the instances' grids row by row (node quads of all
                // instances cost more than they save: four times the grids no longer stay in L2)
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
