// Calculation step of Algorithms 2.1 / 3.1 / 4.1 for many targets: reduce each
// target to the period cell (step 2c), branch on |x_t| <= c (step 2b),
// interpolate the near grid with the tensor-product 4-point Lagrange rule
// (16 / 64 nodes, step 2d), add back the removed singular part in FP64 and apply
// the quasi-periodic phase (steps 2e-2f; Algorithm 4.1 steps 2e-2i).  Far
// targets interpolate the far-slab grid of the eigenfunction series.
#include "qpgf_internal.h"

namespace qpgf {

namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

struct GArgs {
  double k, a1, a2, c, c_tilde, eps, rmin;
  int M1, M2, M3;          // 2D: M2 = transverse size, M3 = 1
  double h1, h2, h3;       // 2D: h2 = transverse spacing
  double hf;               // far-slab spacing
  int S;                   // far-slab slices
  long fs, ffs;            // field strides (near, far)
};

// cubic Lagrange weights at nodes -1, 0, 1, 2
__device__ __forceinline__ void lag4(double f, double w[4]) {
  const double fm1 = f - 1.0, fm2 = f - 2.0, fp1 = f + 1.0;
  w[0] = -f * fm1 * fm2 * (1.0 / 6.0);
  w[1] = fp1 * fm1 * fm2 * 0.5;
  w[2] = -fp1 * f * fm2 * 0.5;
  w[3] = fp1 * f * fm1 * (1.0 / 6.0);
}

// x = 2 pi n + t, t in [-pi, pi)
__device__ __forceinline__ double reduce_cell(double x, double& n) {
  n = floor((x + kPi) / (2.0 * kPi));
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

// sum over the 4 x 4 (x 4) stencil of field f: weights w1 (x1), w2 (x2), w3 (slices)
template <typename T, int NF>
__device__ __forceinline__ void stencil3(const cplx<T>* __restrict__ g, long fs, const int i1[4], const int i2[4],
                                         const long i3[4], const double w1[4], const double w2[4], const double w3[4],
                                         int M1, int M2, double2 out[NF]) {
  Acc<T> acc[NF];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const long row = (i3[c] * M2 + i2[b]) * (long)M1;
      const T wcb = (T)(w3[c] * w2[b]);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const T w = wcb * (T)w1[a];
#pragma unroll
        for (int f = 0; f < NF; ++f) acc[f].add(w, g[f * fs + row + i1[a]]);
      }
    }
  }
#pragma unroll
  for (int f = 0; f < NF; ++f) out[f] = acc[f].get();
}

__device__ __forceinline__ double2 nan2() { return mk(__builtin_nan(""), __builtin_nan("")); }

// 3D: G_d (NF = 1) or the Maxwell tensor (NF = 7, output [T][6]).
template <typename T, int NF>
__global__ __launch_bounds__(256) void k_gather3d(GArgs A, const cplx<T>* __restrict__ grid,
                                                  const cplx<T>* __restrict__ far, const double* __restrict__ x,
                                                  long T_, cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T_) return;
  const double x1 = x[3 * i], x2 = x[3 * i + 1], x3 = x[3 * i + 2];
  constexpr int NO = (NF == 1) ? 1 : 6;
  uint8_t fl = 0;
  double2 res[NO];
  if (!(isfinite(x1) && isfinite(x2) && isfinite(x3))) {
    fl = 8;
#pragma unroll
    for (int o = 0; o < NO; ++o) res[o] = nan2();
  } else {
    double n1, n2;
    const double t1 = reduce_cell(x1, n1), t2 = reduce_cell(x2, n2);
    double w1[4], w2[4], w3[4];
    int i1[4], i2[4];
    long i3[4];
    {
      const double u = t1 / A.h1, p = floor(u);
      lag4(u - p, w1);
#pragma unroll
      for (int a = 0; a < 4; ++a) i1[a] = ((int)p - 1 + a) & (A.M1 - 1);
    }
    {
      const double u = t2 / A.h2, p = floor(u);
      lag4(u - p, w2);
#pragma unroll
      for (int a = 0; a < 4; ++a) i2[a] = ((int)p - 1 + a) & (A.M2 - 1);
    }
    double ps, pc;
    sincos(A.a1 * x1 + A.a2 * x2, &ps, &pc);
    const double2 phase = mk(pc, ps);
    double2 L[NF];
    const bool is_near = fabs(x3) <= A.c;
    bool bad = false;
    if (is_near) {
      const double u = x3 / A.h3, p = floor(u);
      lag4(u - p, w3);
#pragma unroll
      for (int a = 0; a < 4; ++a) i3[a] = ((int)p - 1 + a) & (A.M3 - 1);
      stencil3<T, NF>(grid, A.fs, i1, i2, i3, w1, w2, w3, A.M1, A.M2, L);
    } else {
      fl |= 2;
      const double v = (fabs(x3) - (A.c - A.hf)) / A.hf;
      double s0 = floor(v);
      if (s0 > A.S - 3) {
        bad = true;
        fl |= 4;
      } else {
        s0 = fmax(s0, 1.0);
        lag4(v - s0, w3);
#pragma unroll
        for (int a = 0; a < 4; ++a) i3[a] = (long)s0 - 1 + a;
        stencil3<T, NF>(far, A.ffs, i1, i2, i3, w1, w2, w3, A.M1, A.M2, L);
      }
    }
    if (bad) {
#pragma unroll
      for (int o = 0; o < NO; ++o) res[o] = nan2();
    } else {
      double2 G[NF];
#pragma unroll
      for (int f = 0; f < NF; ++f) G[f] = cmul(phase, L[f]);
      if (!is_near && NF == 7) {
        // d/dx3 of e^{i beta |x3|} carries sgn(x3): components 13 and 23
        if (x3 < 0) { G[5] = cscale(G[5], -1.0); G[6] = cscale(G[6], -1.0); }
      }
      if (is_near) {
        const double r = sqrt(t1 * t1 + t2 * t2 + x3 * x3);
        if (r <= A.rmin || r == 0.0) {
          fl |= 1;
#pragma unroll
          for (int f = 0; f < NF; ++f) G[f] = nan2();
        } else if (r < 2.0 * A.eps) {
          // psi = e^{ikr} Y(r) / (4 pi r): the removed singular part F, times e^{i alpha.x'}
          double sn, cn;
          sincos(A.k * r, &sn, &cn);
          const double2 g = cscale(mk(cn, sn), 1.0 / (4.0 * kPi * r));
          const double2 lat = [&] {
            double ls, lc;
            sincospi(2.0 * (A.a1 * n1 + A.a2 * n2), &ls, &lc);
            return mk(lc, ls);
          }();
          const double Y = cut_Y(r, A.eps);
          G[0] = cadd(G[0], cmul(lat, cscale(g, Y)));
          if (NF == 7) {
            // psi' and psi'' (radial), then d_p d_q psi = psi'' t_p t_q / r^2 + psi' (delta_pq / r - t_p t_q / r^3)
            const double Y1 = cut_Y1(r, A.eps), Y2 = cut_Y2(r, A.eps);
            const double2 ikr = mk(-1.0 / r, A.k);                 // ik - 1/r
            const double2 g1 = cmul(g, ikr);
            const double2 g2 = cmul(g, cadd(cmul(ikr, ikr), mk(1.0 / (r * r), 0.0)));
            const double2 d1 = cadd(cscale(g1, Y), cscale(g, Y1));
            const double2 d2 = cadd(cadd(cscale(g2, Y), cscale(g1, 2.0 * Y1)), cscale(g, Y2));
            const double t[3] = {t1, t2, x3};
            const int P[6] = {0, 1, 2, 0, 0, 1}, Qp[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
            for (int f = 0; f < 6; ++f) {
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
        // GG_pq = delta_pq G_d + k^-2 d_p d_q G_d  (eq. 4.1)
        const double ik2 = 1.0 / (A.k * A.k);
#pragma unroll
        for (int f = 0; f < 6; ++f) {
          double2 v = cscale(G[f + 1], ik2);
          if (f < 3) v = cadd(v, G[0]);
          res[f] = v;
        }
      }
    }
  }
#pragma unroll
  for (int o = 0; o < NO; ++o) store_out<T>(out, i * NO + o, res[o]);
  if (flags) flags[i] = fl;
}

// 2D: G (Algorithm 2.1).
template <typename T>
__global__ __launch_bounds__(256) void k_gather2d(GArgs A, const cplx<T>* __restrict__ grid,
                                                  const cplx<T>* __restrict__ far, const double* __restrict__ x,
                                                  long T_, cplx<T>* __restrict__ out, uint8_t* __restrict__ flags) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= T_) return;
  const double x1 = x[2 * i], x2 = x[2 * i + 1];
  uint8_t fl = 0;
  double2 res;
  if (!(isfinite(x1) && isfinite(x2))) {
    fl = 8;
    res = nan2();
  } else {
    double n1;
    const double t = reduce_cell(x1, n1);
    double w1[4], w2[4];
    int i1[4];
    {
      const double u = t / A.h1, p = floor(u);
      lag4(u - p, w1);
#pragma unroll
      for (int a = 0; a < 4; ++a) i1[a] = ((int)p - 1 + a) & (A.M1 - 1);
    }
    double ps, pc;
    sincos(A.a1 * x1, &ps, &pc);
    const double2 phase = mk(pc, ps);
    const bool is_near = fabs(x2) <= A.c;
    long rows[4];
    const cplx<T>* g = grid;
    bool bad = false;
    if (is_near) {
      const double u = x2 / A.h2, p = floor(u);
      lag4(u - p, w2);
#pragma unroll
      for (int b = 0; b < 4; ++b) rows[b] = (long)(((int)p - 1 + b) & (A.M2 - 1)) * A.M1;
    } else {
      fl |= 2;
      g = far;
      const double v = (fabs(x2) - (A.c - A.hf)) / A.hf;
      double s0 = floor(v);
      if (s0 > A.S - 3) {
        bad = true;
        fl |= 4;
      } else {
        s0 = fmax(s0, 1.0);
        lag4(v - s0, w2);
#pragma unroll
        for (int b = 0; b < 4; ++b) rows[b] = ((long)s0 - 1 + b) * A.M1;
      }
    }
    if (bad) {
      res = nan2();
    } else {
      Acc<T> acc;
#pragma unroll
      for (int b = 0; b < 4; ++b)
#pragma unroll
        for (int a = 0; a < 4; ++a) acc.add((T)(w2[b] * w1[a]), g[rows[b] + i1[a]]);
      double2 Lt = acc.get();
      if (is_near) {
        const double r = sqrt(t * t + x2 * x2);
        if (r <= A.rmin || r == 0.0) {
          fl |= 1;
          Lt = nan2();
        } else if (r < 2.0 * A.eps) {
          // K_N = L_N + f1 - i alpha f2 = L_N - (1/2pi) ln r Y(r) (1 - i alpha t)
          const double s = -log(r) * cut_Y(r, A.eps) / (2.0 * kPi);
          Lt = cadd(Lt, mk(s, -A.a1 * t * s));
        }
      }
      res = cmul(phase, Lt);
    }
  }
  store_out<T>(out, i, res);
  if (flags) flags[i] = fl;
}

template <typename T>
hipError_t gather_impl(Plan& P, const double* x, int64_t T_, void* out, uint8_t* flags) {
  GArgs A;
  A.k = P.last_k;
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
  A.hf = P.p.far_h;
  A.S = P.S;
  A.fs = (long)P.ncell;
  A.ffs = (long)P.nfar;
  const auto* g = static_cast<const cplx<T>*>(P.grid);
  const auto* f = static_cast<const cplx<T>*>(P.far);
  auto* o = static_cast<cplx<T>*>(out);
  const dim3 grid((unsigned)((T_ + 255) / 256));
  if (P.dim == 2)
    hipLaunchKernelGGL(k_gather2d<T>, grid, dim3(256), 0, P.stream, A, g, f, x, (long)T_, o, flags);
  else if (P.nf == 7)
    hipLaunchKernelGGL((k_gather3d<T, 7>), grid, dim3(256), 0, P.stream, A, g, f, x, (long)T_, o, flags);
  else
    hipLaunchKernelGGL((k_gather3d<T, 1>), grid, dim3(256), 0, P.stream, A, g, f, x, (long)T_, o, flags);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gather(Plan& P, const double* x, int64_t T_, void* out, uint8_t* flags) {
  if (T_ <= 0) return hipSuccess;
  return P.p.prec == QPGF_C128 ? gather_impl<double>(P, x, T_, out, flags) : gather_impl<float>(P, x, T_, out, flags);
}

}  // namespace qpgf
