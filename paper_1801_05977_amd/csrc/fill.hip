// FP64 coefficient fills: L-hat of the near grid (2D: eqs. 2.1, 2.3-2.5;
// 3D: eqs. 3.3, 3.5; Maxwell: Section 4), the k-independent 2D singular tables
// (eqs. 2.4, 2.5), the radial table of the 3D singular transform, and the
// far-slab coefficients of the eigenfunction series (1.2), (1.3).
//
// Layout: coefficient j (centred, -M/2 <= j < M/2) of an axis of size M is
// stored at index j mod M ("FFT order"), so the grid sums become plain
// unnormalised inverse DFTs.  Near fields: [jt'][j2'][j1'] (3D) or [j2'][j1']
// (2D), j1 fastest; far slab: [s][j2'][j1'] or [s][j1'].
#include "fft_device.h"
#include "qpgf_internal.h"

namespace qpgf {

namespace {

constexpr int TP = 16;   // pencils (periodic-axis coefficients) per block
constexpr int TL = 16;   // transverse lanes per pencil
constexpr double kPi = 3.141592653589793238462643383279502884;

__device__ __forceinline__ int centered(int jp, int M) { return jp < (M >> 1) ? jp : jp - M; }

template <typename T> __device__ __forceinline__ void store_c(cplx<T>* p, size_t i, double2 v);
template <> __device__ __forceinline__ void store_c<double>(double2* p, size_t i, double2 v) { p[i] = v; }
template <> __device__ __forceinline__ void store_c<float>(float2* p, size_t i, double2 v) {
  p[i] = make_float2((float)v.x, (float)v.y);
}

struct FillArgs {
  double k, a1, a2;
  double k2;                 // second wavenumber (differences of second derivatives, 2D)
  double c, c_tilde, A;      // A = A2 = 1/(2 sqrt(pi c~)) or A3 = 1/sqrt(8 pi^2 c~)
                             // (the basis normalisation: L-hat carries one factor A,
                             // the grid sum L_N = sum L-hat_j phi_j another; both are
                             // applied here so the FFTs are plain sums)
  int M1, M2, Mt, Q;
  int Qr;                    // nodes of the radial rule
  double hd;                 // H table spacing (3D)
  long fstride;              // elements per field
  // special coefficients (a propagating beta within stol of |J|, Sections 2.1 / 3.1)
  double stol;
  const double* wXq;         // w_q X(x_q) at the X'-rule nodes on [c, (c + c~)/2]
  const double* rq;          // radial rule on [eps, 2 eps] (3D singular part)
  const double* wrq;
  double eps;
  // 2D G: tables of the removed degree-2 and degree-3 terms (Remark 5.3), nullptr for sing_order 1
  const double* E;
  int sing_order;
};

// a_q = w_q X'(x_q) e^{i beta x_q} for the TP pencils of this block, into LDS.
// beta depends on the pencil only, so the X'-integrals of every transverse
// coefficient of a pencil reduce to sums over these Q values.
template <int DIM>
__device__ __forceinline__ void pencil_weights(const FillArgs& A, int j1p0, int j2p, const double* __restrict__ xq,
                                               const double* __restrict__ wxq, double2* sa) {
  for (int idx = threadIdx.x; idx < TP * A.Q; idx += blockDim.x) {
    int pp = idx / A.Q, q = idx - pp * A.Q;
    int j1p = min(j1p0 + pp, A.M1 - 1);
    double rho;
    if (DIM == 2) {
      rho = fabs(A.a1 + centered(j1p, A.M1));
    } else {
      double e1 = A.a1 + centered(j1p, A.M1), e2 = A.a2 + centered(j2p, A.M2);
      rho = sqrt(e1 * e1 + e2 * e2);
    }
    double2 b = beta_of(A.k, rho);
    // [q][pencil]: the 16 pencils of a wave read 16 consecutive entries
    sa[q * TP + pp] = cscale(cexpi(cscale(b, xq[q])), wxq[q]);
  }
}

// I(b - J)/(2b(J - b)) - I(b + J)/(2b(J + b)), with I(g) = int e^{igx} X'(x) dx
// = sum_q a_q e^{-+iJx_q}:  I(b-J) = C - iS, I(b+J) = C + iS,
// C = sum_q a_q cos(J x_q), S = sum_q a_q sin(J x_q).
__device__ __forceinline__ double2 xprime_term(const double2* __restrict__ ap, const double2* __restrict__ csr, int Q,
                                               double sgn, double J, double2 b) {
  double2 C = mk(0.0, 0.0), S = mk(0.0, 0.0);
#pragma unroll 8
  for (int q = 0; q < Q; ++q) {
    double2 a = ap[q * TP], t = csr[q];
    C.x = fma(a.x, t.x, C.x);
    C.y = fma(a.y, t.x, C.y);
    S.x = fma(a.x, t.y, S.x);
    S.y = fma(a.y, t.y, S.y);
  }
  S = cscale(S, sgn);
  double2 Im = mk(C.x + S.y, C.y - S.x);
  double2 Ip = mk(C.x - S.y, C.y + S.x);
  double2 b2 = cscale(b, 2.0);
  double2 dm = cmul(b2, mk(J - b.x, -b.y));
  double2 dp = cmul(b2, mk(J + b.x, b.y));
  return csub(cdiv(Im, dm), cdiv(Ip, dp));
}

// ---- special coefficients: beta = -+J (Sections 2.1 / 3.1) ----
// There the integration by parts behind (2.1) / (3.3) divides by beta -+ J (and loses digits
// close to it); the coefficient is taken from the integral that defines it,
//   K-hat_j / A = (i / (2 beta)) [I0(beta - J) + I0(beta + J)],   I0(g) = int_0^{c~} e^{igx} X(x) dx,
// the paper's special-case formula (its g = 0 term is int X) for every g near the special point.
// The fills compute every coefficient by the integrated form in their main loop and then
// overwrite a pencil's (at most two) special ones, so the loop is the same as without them.

// The FFT-order transverse indices of the (at most two) special coefficients of a pencil:
// jt = +-js with |beta - js pi / c~| < stol for a propagating beta; -1 where there is none.
// special_tol < pi / (4 c~) (checked at plan creation), so js is unique.
__device__ __forceinline__ void special_jts(double2 b, const FillArgs& A, int js_idx[2]) {
  js_idx[0] = js_idx[1] = -1;
  if (b.y != 0.0) return;
  const double step = kPi / A.c_tilde;
  const int js = (int)rint(b.x / step);
  if (js > A.Mt / 2 || !(fabs(b.x - js * step) < A.stol)) return;
  js_idx[0] = js & (A.Mt - 1);
  js_idx[1] = (-js) & (A.Mt - 1);
  if (js_idx[1] == js_idx[0]) js_idx[1] = -1;
}
// (e^{i th} - 1) / (i th), without cancellation for small th
__device__ __forceinline__ double2 e1i(double th) {
  if (th == 0.0) return mk(1.0, 0.0);
  const double h = sin(0.5 * th);
  return mk(sin(th) / th, 2.0 * h * h / th);
}
// I0(g) = c E1(i g c) + sum_q w_q X(x_q) e^{i g x_q}  (X = 1 on [0, c], 0 beyond (c + c~)/2)
__device__ double2 x_integral0(double g, const FillArgs& A, const double* __restrict__ xq) {
  double2 s = cscale(e1i(g * A.c), A.c);
  for (int q = 0; q < A.Q; ++q) {
    double sn, cn;
    sincos(g * xq[q], &sn, &cn);
    s.x = fma(A.wXq[q], cn, s.x);
    s.y = fma(A.wXq[q], sn, s.y);
  }
  return s;
}
__device__ double2 khat_direct(double beta, double J, const FillArgs& A, const double* __restrict__ xq) {
  const double2 I = cadd(x_integral0(beta - J, A, xq), x_integral0(beta + J, A, xq));
  return cmul(mk(0.0, 0.5 / beta), I);
}
// 3D: at |xi| = k the singular part's coefficient (1 - H)/(|xi|^2 - k^2) is 0/0; its value is
// the radial transform of e^{ikr} Y / (4 pi r), (1/rho) int_0^{2 eps} e^{ikr} Y(r) sin(rho r) dr:
// closed form on [0, eps] (Y = 1), the radial rule on [eps, 2 eps].
__device__ double2 fhat_direct(double k, double rho, const FillArgs& A) {
  const double e = A.eps;
  // int_0^eps e^{ikr} sin(rho r) dr = (eps / 2i) [E1(i(k + rho) eps) - E1(i(k - rho) eps)]
  const double2 d = csub(e1i((k + rho) * e), e1i((k - rho) * e));
  double2 s = mk(0.5 * e * d.y, -0.5 * e * d.x);
  for (int q = 0; q < A.Qr; ++q) {
    const double r = A.rq[q];
    double sn, cn;
    sincos(k * r, &sn, &cn);
    const double w = A.wrq[q] * cut_Y(r, e) * sin(rho * r);
    s.x = fma(w, cn, s.x);
    s.y = fma(w, sn, s.y);
  }
  return cscale(s, 1.0 / rho);
}

// H(rho) by 8-point Lagrange interpolation of the table H(m hd - 4 hd).
__device__ __forceinline__ double2 h_interp(const double2* __restrict__ tab, double hd, double rho) {
  double u = rho / hd;
  double fl = floor(u);
  double f = u - fl;
  int m0 = (int)fl + 1;   // table index of the node at relative position -3
  double pre[8], suf[8];
  pre[0] = 1.0;
#pragma unroll
  for (int a = 1; a < 8; ++a) pre[a] = pre[a - 1] * (f - (double)(a - 4));
  suf[7] = 1.0;
#pragma unroll
  for (int a = 6; a >= 0; --a) suf[a] = suf[a + 1] * (f - (double)(a - 2));
  // reciprocals of the node products prod_{b != a} (a - b) for nodes -3..4
  const double rden[8] = {-1.0 / 5040.0, 1.0 / 720.0, -1.0 / 240.0, 1.0 / 144.0,
                          -1.0 / 144.0,  1.0 / 240.0, -1.0 / 720.0, 1.0 / 5040.0};
  double2 acc = mk(0.0, 0.0);
#pragma unroll
  for (int a = 0; a < 8; ++a) {
    double w = pre[a] * suf[a] * rden[a];
    double2 h = tab[m0 + a];
    acc.x = fma(w, h.x, acc.x);
    acc.y = fma(w, h.y, acc.y);
  }
  return acc;
}

// 3D near fill (Algorithm 3.1 steps 1a-1b; Algorithm 4.1 step 1c when NF is kMxF or kMxT):
// L-hat_dj = A3 [ I-terms + H(|xi|) / (|xi|^2 - k^2) ], i.e. K-hat_dj of (3.3)
// minus F-hat_j of (3.5) with the common 1/(|xi|^2-k^2) cancelled exactly.
//
// FUSE: the block also runs the transverse inverse DFT of its TP pencils of
// every field (Algorithm 3.1 step 1c; the NF fields of the Maxwell kinds) in
// LDS and writes grid values instead of coefficients, saving one pass over the
// grid (the transform is the same sequence of passes and twiddles as the
// separate FFT kernel).
template <typename T, int NF, bool FUSE, bool SPEC>
__global__ __launch_bounds__(256) void k_fill3d(FillArgs A, const double* __restrict__ xq,
                                                const double* __restrict__ wxq, const double2* __restrict__ cs,
                                                const double2* __restrict__ htab, cplx<T>* __restrict__ out,
                                                const cplx<T>* __restrict__ tw, int ntw) {
  extern __shared__ double2 sa[];
  // FUSE: the pencils, [field][pencil][jt'] with pitch Mt + 1, after the weights
  cplx<T>* pen = reinterpret_cast<cplx<T>*>(sa + TP * A.Q);
  const int pitch = A.Mt + 1;
  const int ip = threadIdx.x % TP, lane = threadIdx.x / TP;
  const int j1p0 = blockIdx.x * TP, j2p = blockIdx.y;
  const int j1p = j1p0 + ip;
  const double xi1 = A.a1 + centered(min(j1p, A.M1 - 1), A.M1), xi2 = A.a2 + centered(j2p, A.M2);
  const double rp2 = xi1 * xi1 + xi2 * xi2;
  const double2 b = beta_of(A.k, sqrt(rp2));
  const bool use_I = b.y * A.c < 41.5;   // else |I| < e^{-c Im beta} < 1e-18
  // the pencil weights only where some pencil of the block needs the X'-integrals
  if (__syncthreads_or(use_I && j1p < A.M1)) pencil_weights<3>(A, j1p0, j2p, xq, wxq, sa);
  __syncthreads();
  if (!FUSE && j1p >= A.M1) return;
  const double2* ap = sa + ip;
  const double k2 = A.k * A.k;
  // coefficient jt' of this pencil: into the LDS pencil (FUSE) or the near grid (and the Maxwell fields)
  auto put = [&](int jtp, double J, double2 L) {
    // field g of coefficient jt': the LDS pencil (FUSE) or the near grid
    auto put1 = [&](int g, double2 v) {
      if constexpr (FUSE) store_c<T>(pen, ((size_t)g * TP + ip) * pitch + jtp, v);
      else store_c<T>(out, g * A.fstride + ((size_t)jtp * A.M2 + j2p) * A.M1 + j1p, v);
    };
    put1(0, L);
    if constexpr (NF == kMxF || NF == kMxT) {
      // L-hat^{pq} = -c^p c^q L-hat with c = (alpha1 + j1, alpha2 + j2, j3 pi / c~) (Algorithm 4.1 step 1c),
      // pq = 11 22 33 12 13 23 (without 33 for the trace variant)
      const double cc[3] = {xi1, xi2, J};
      constexpr int NP = NF - 1;
      const int P[6] = {0, 1, 2, 0, 0, 1}, Qp[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
      for (int f = 0, g = 0; f < 6; ++f) {
        if (NP == 5 && f == 2) continue;
        put1(++g, cscale(L, -cc[P[f]] * cc[Qp[f]]));
      }
    }
  };
  for (int jtp = lane; jtp < A.Mt; jtp += TL) {
    const int jt = centered(jtp, A.Mt);
    const double J = jt * kPi / A.c_tilde;
    double2 term = mk(0.0, 0.0);
    if (use_I) term = xprime_term(ap, cs + (size_t)abs(jt) * A.Q, A.Q, jt < 0 ? -1.0 : 1.0, J, b);
    const double rho2 = rp2 + J * J;
    const double2 H = h_interp(htab, A.hd, sqrt(rho2));
    put(jtp, J, cscale(cadd(term, cscale(H, 1.0 / (rho2 - k2))), A.A * A.A));
  }
  if constexpr (SPEC) {
    // the special coefficients of this pencil, recomputed over what the loop wrote:
    // L-hat = K-hat - F-hat, each from its defining integral
    int js[2];
    special_jts(b, A, js);
    for (int s = 0; s < 2; ++s) {
      if (js[s] < 0 || j1p >= A.M1 || js[s] % TL != lane) continue;
      const double J = centered(js[s], A.Mt) * kPi / A.c_tilde;
      const double rho = sqrt(rp2 + J * J);
      put(js[s], J, cscale(csub(khat_direct(b.x, J, A, xq), fhat_direct(A.k, rho, A)), A.A * A.A));
    }
  }
  if constexpr (FUSE) {
    __syncthreads();
    fftdev::inverse_dft_lds<T>(pen, A.Mt, pitch, TP * NF, tw, ntw);
    // grid values [field][i3][j2'][j1'], TP consecutive j1' per slice
    const int np = min(TP, A.M1 - j1p0);
    for (int idx = threadIdx.x; idx < NF * TP * A.Mt; idx += blockDim.x) {
      const int p = idx % TP, r = idx / TP, i3 = r % A.Mt, g = r / A.Mt;
      if (p < np) out[g * A.fstride + ((size_t)i3 * A.M2 + j2p) * A.M1 + j1p0 + p] = pen[(g * TP + p) * pitch + i3];
    }
  }
}

// 2D near fill (Algorithm 2.1 steps 1a-1b): L-hat = K-hat (2.1) - F1 + i alpha F2 (2.3).
// F1, F2: singular tables for x1 size M1t >= A.M1 (entry j at j mod M1t), shared by
// every instance whose x1 size divides into the same table.
template <typename T, bool SPEC>
__device__ __forceinline__ void fill2d_body(const FillArgs& A, int blk, const double* __restrict__ xq,
                                            const double* __restrict__ wxq, const double2* __restrict__ cs,
                                            const double2* __restrict__ F1, const double2* __restrict__ F2, int M1t,
                                            cplx<T>* __restrict__ out, double2* sa) {
  const int ip = threadIdx.x % TP, lane = threadIdx.x / TP;
  const int j1p0 = blk * TP;
  const int j1p = j1p0 + ip;
  const int j1 = centered(min(j1p, A.M1 - 1), A.M1);
  const double a = A.a1 + j1;
  const double2 b = beta_of(A.k, fabs(a));
  const bool use_I = b.y * A.c < 41.5;
  if (__syncthreads_or(use_I && j1p < A.M1)) pencil_weights<2>(A, j1p0, 0, xq, wxq, sa);
  __syncthreads();
  if (j1p >= A.M1) return;
  const double2* ap = sa + ip;
  const double lead0 = a * a - A.k * A.k;
  const int jt_tab = j1 < 0 ? j1 + M1t : j1;
  // E-hat = -(alpha^2/2) e_tt - (k^2/4) e_rr - (alpha^3/6) e_ttt - (alpha k^2/4) e_trr (real)
  const double ka = A.k * A.k;
  const double ce0 = -0.5 * A.a1 * A.a1, ce1 = -0.25 * ka;
  const double ce2 = A.sing_order >= 3 ? -A.a1 * A.a1 * A.a1 / 6.0 : 0.0;
  const double ce3 = A.sing_order >= 3 ? -0.25 * A.a1 * ka : 0.0;
  const size_t en = (size_t)A.Mt * M1t;
  auto put = [&](int jtp, double2 K) {
    const size_t ot = (size_t)jtp * M1t + jt_tab;
    const double2 f1 = F1[ot], f2 = F2[ot];
    // L = K - F1 + i alpha F2 (- E-hat), times the basis normalisation A2
    double lx = K.x - f1.x - A.a1 * f2.y;
    if (A.E) {
      const double* e = A.E + ot;
      lx -= ce0 * e[0] + ce1 * e[en] + ce2 * e[2 * en] + ce3 * e[3 * en];
    }
    const double2 L = cscale(mk(lx, K.y - f1.y + A.a1 * f2.x), A.A);
    store_c<T>(out, (size_t)jtp * A.M1 + j1p, L);
  };
  for (int jtp = lane; jtp < A.Mt; jtp += TL) {
    const int jt = centered(jtp, A.Mt);
    const double J = jt * kPi / A.c_tilde;
    double2 term = mk(0.0, 0.0);
    if (use_I) term = xprime_term(ap, cs + (size_t)abs(jt) * A.Q, A.Q, jt < 0 ? -1.0 : 1.0, J, b);
    put(jtp, cscale(cadd(term, mk(1.0 / (lead0 + J * J), 0.0)), A.A));
  }
  if constexpr (SPEC) {
    // the special coefficients of this pencil, recomputed from their defining integral
    int js[2];
    special_jts(b, A, js);
    for (int s = 0; s < 2; ++s) {
      if (js[s] < 0 || js[s] % TL != lane) continue;
      put(js[s], cscale(khat_direct(b.x, centered(js[s], A.Mt) * kPi / A.c_tilde, A, xq), A.A));
    }
  }
}

template <typename T, bool SPEC>
__global__ __launch_bounds__(256) void k_fill2d(FillArgs A, const double* __restrict__ xq,
                                                const double* __restrict__ wxq, const double2* __restrict__ cs,
                                                const double2* __restrict__ F1, const double2* __restrict__ F2,
                                                cplx<T>* __restrict__ out) {
  extern __shared__ double2 sa[];
  fill2d_body<T, SPEC>(A, blockIdx.x, xq, wxq, cs, F1, F2, A.M1, out, sa);
}

// Many 2D instances in one launch: instance i owns blocks [inst[i].blk0, inst[i+1].blk0).
struct FillInst {
  FillArgs A;
  int Mf1, Sf;   // modes and slices of the instance's far slab
  double hf, z0; // its slice spacing and first slice
  long off;      // first element of the instance's near grid
  long foff;     // first element of its far slab
  long blk0;     // first block of the instance in this launch
};

__device__ __forceinline__ int find_inst(const FillInst* __restrict__ inst, int n, long blk) {
  int lo = 0, hi = n - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (inst[mid].blk0 <= blk) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T, bool SPEC>
__global__ __launch_bounds__(256) void k_fill2d_multi(const FillInst* __restrict__ inst, int n_inst,
                                                      const double* __restrict__ xq, const double* __restrict__ wxq,
                                                      const double2* __restrict__ cs, const double2* __restrict__ F1,
                                                      const double2* __restrict__ F2, int M1t,
                                                      cplx<T>* __restrict__ base) {
  extern __shared__ double2 sa[];
  const int i = find_inst(inst, n_inst, blockIdx.x);
  const FillInst I = inst[i];
  fill2d_body<T, SPEC>(I.A, (int)(blockIdx.x - I.blk0), xq, wxq, cs, F1, F2, M1t, base + I.off, sa);
}

// 2D singular tables (eqs. 2.4, 2.5), k- and alpha-independent (Remark 2.1):
// Phi-hat_1 / 2pi = A2 int Phi1(r) J0(|eta| r) r dr,
// Phi-hat_2 / 2pi = -i A2 (j1/|eta|) int Phi1(r) J1(|eta| r) r^2 dr, eta = (j1, j2 pi/c~).
__global__ void k_sing2d(int M1, int M2, double c_tilde, double A2, int Q, const double* __restrict__ rq,
                         const double* __restrict__ wphi, double f1zero, double2* __restrict__ F1,
                         double2* __restrict__ F2) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M1 * M2) return;
  const int j1p = (int)(idx % M1), j2p = (int)(idx / M1);
  const double e1 = centered(j1p, M1), J = centered(j2p, M2) * kPi / c_tilde;
  const double eta2 = e1 * e1 + J * J;
  if (eta2 == 0.0) {
    F1[idx] = mk(f1zero, 0.0);
    F2[idx] = mk(0.0, 0.0);
    return;
  }
  const double eta = sqrt(eta2);
  double i0 = 0.0, i1 = 0.0;
  for (int q = 0; q < Q; ++q) {
    const double r = rq[q], er = eta * r;
    i0 = fma(wphi[q] * r, j0(er), i0);
    i1 = fma(wphi[q] * r * r, j1(er), i1);
  }
  const double f1 = (A2 + A2 * i0) / eta2;
  F1[idx] = mk(f1, 0.0);
  F2[idx] = mk(0.0, (-2.0 * e1 * f1 - A2 * (e1 / eta) * i1) / eta2);
}

// Gradient tables (Section 2.4.1): the Fourier coefficients of the singular parts
//   h1 = -(1/2pi) [-(k^2/2) x1 ln r + x1/r^2 - i alpha x1^2/r^2 - (alpha^2/2) x1^3/r^2] Y(r),
//   h2 = -(1/2pi) [-(k^2/2) x2 ln r + x2/r^2 - i alpha x1 x2/r^2 - (alpha^2/2) x1^2 x2/r^2] Y(r)
// split by their k- and alpha-dependence, H-hat_p = i (k^2 a_p + P_p - alpha Q_p - (alpha^2/2) R_p),
// so the eight real tables a1 P1 Q1 R1 a2 P2 Q2 R2 ([8][M2][M1], A2 included) serve every
// (k, alpha).  Each term is a radial function times cos(n theta) or sin(n theta); its
// coefficient is 2 pi (-i)^n cos(n phi) (or sin) times int g(r) J_n(|eta| r) r dr, phi the angle
// of eta = (j1, j2 pi / c~).  Y = 1 on [0, eps], where the six radial integrals have closed
// forms (recurrences and d/dz[z^n J_n] = z^n J_{n-1}); on [eps, 2 eps] a Gauss-Legendre rule
// (weights times Y at the nodes) fine enough for the highest |eta| of the grid.
// Radial integrals of the singular parts' coefficients at |eta| = rho > 0, over [0, 2 eps]:
//   TA = int ln r Y J1 r^2,  TB = int Y J1,  TC0 = int Y J0 r,  TC2 = int Y J2 r,
//   TD1 = int Y J1 r^2,  TD3 = int Y J3 r^2,  TL = int ln r Y J0 r   (dr).
// Y = 1 on [0, eps], where they have closed forms (the recurrence of J_n, d/dz[z^n J_n] =
// z^n J_{n-1}, integration by parts for the ln r ones); on [eps, 2 eps] a Gauss-Legendre rule
// whose weights carry Y at the nodes.
struct Radial {
  double TA, TB, TC0, TC2, TD1, TD3, TL;
};

// Higher-order 2D tables (Remark 5.3): the Fourier coefficients of the degree-2 and
// degree-3 terms of the removed -(1/2pi) ln r Y(r) P_m(x1, r),
//   -(alpha^2/2) x1^2 - (k^2/4) r^2 + i (alpha^3/6) x1^3 + i (alpha k^2/4) x1 r^2,
// split by their k- and alpha-dependence into four real tables ([4][M2][M1], A2 and -1/2pi
// included): e_tt (x1^2 ln r), e_rr (r^2 ln r) and the imaginary parts e_ttt (x1^3 ln r),
// e_trr (x1 r^2 ln r), so that E-hat = -(alpha^2/2) e_tt - (k^2/4) e_rr - (alpha^3/6) e_ttt
// - (alpha k^2/4) e_trr.  With x1^2 = r^2 (1 + cos 2 theta)/2, x1^3 = r^3 (3 cos theta +
// cos 3 theta)/4 and the plane-wave expansion (a radial g times cos n theta has the
// coefficient 2 pi (-i)^n cos n phi int g J_n(|eta| r) r dr), four radial integrals serve:
//   T03 = int r^3 ln r Y J0,  T23 = int r^3 ln r Y J2,  T14 = int r^4 ln r Y J1,  T34 = int r^4 ln r Y J3.
// On [0, eps] (Y = 1) integration by parts against the antiderivatives int z^3 J0 = z^3 J1 -
// 2 z^2 J2, int z^{n+1} J_n = z^{n+1} J_{n+1}, int z^4 J1 = z^4 J2 - 2 z^3 J3 and the closed
// forms of int z J2, int z^2 J3, int z^3 J4 gives them exactly; on [eps, 2 eps] the
// Gauss-Legendre rule of the derivative tables.
__global__ void k_sing2d_ho(int M1, int M2, double c_tilde, double A2, double eps, int Qg,
                            const double* __restrict__ rg, const double* __restrict__ wyg, double* __restrict__ E) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long n = (long)M1 * M2;
  if (idx >= n) return;
  const int j1p = (int)(idx % M1), j2p = (int)(idx / M1);
  const double e1 = centered(j1p, M1), J = centered(j2p, M2) * kPi / c_tilde;
  const double rho2 = e1 * e1 + J * J;
  const double le = log(eps), e2 = eps * eps, e3 = e2 * eps, e4 = e3 * eps;
  if (rho2 == 0.0) {
    // |eta| = 0: only J0 survives; int_0^eps r^3 ln r dr = eps^4 (ln eps / 4 - 1/16)
    double T03 = e4 * (0.25 * le - 0.0625);
    for (int q = 0; q < Qg; ++q) {
      const double r = rg[q];
      T03 = fma(wyg[q] * r * r * r, log(r), T03);
    }
    E[idx] = -0.5 * A2 * T03;
    E[n + idx] = -A2 * T03;
    E[2 * n + idx] = 0.0;
    E[3 * n + idx] = 0.0;
    return;
  }
  const double rho = sqrt(rho2), ir = 1.0 / rho, ze = rho * eps;
  const double J0e = j0(ze), J1e = j1(ze), J2e = jn(2, ze), J3e = jn(3, ze), J4e = jn(4, ze);
  // int_0^eps r J2 and int_0^eps r^2 J3 (as in the derivative tables)
  const double c2 = 2.0 * (1.0 - J0e) * ir * ir - eps * J1e * ir;
  const double d3 = 4.0 * ir * c2 - e2 * J2e * ir;
  double T03 = le * (e3 * J1e * ir - 2.0 * e2 * J2e * ir * ir) - e2 * J2e * ir * ir + 2.0 * c2 * ir * ir;
  double T23 = le * e3 * J3e * ir - d3 * ir;
  double T14 = le * (e4 * J2e * ir - 2.0 * e3 * J3e * ir * ir) - e3 * J3e * ir * ir + 2.0 * d3 * ir * ir;
  double T34 = le * e4 * J4e * ir - (6.0 * d3 * ir - e3 * J3e * ir) * ir;
  for (int q = 0; q < Qg; ++q) {
    const double r = rg[q], z = rho * r;
    const double w3 = wyg[q] * r * r * r * log(r), w4 = w3 * r;
    T03 = fma(w3, j0(z), T03);
    T23 = fma(w3, jn(2, z), T23);
    T14 = fma(w4, j1(z), T14);
    T34 = fma(w4, jn(3, z), T34);
  }
  const double cp = e1 * ir, c2p = (e1 * e1 - J * J) / rho2, c3p = cp * (4.0 * cp * cp - 3.0);
  E[idx] = -0.5 * A2 * (T03 - c2p * T23);
  E[n + idx] = -A2 * T03;
  E[2 * n + idx] = 0.25 * A2 * (3.0 * cp * T14 - c3p * T34);
  E[3 * n + idx] = A2 * cp * T14;
}
__device__ Radial radial_integrals(double rho, double eps, int Qg, const double* __restrict__ rg,
                                   const double* __restrict__ wyg) {
  const double ze = rho * eps, J0e = j0(ze), J1e = j1(ze), J2e = jn(2, ze), ir = 1.0 / rho, le = log(eps);
  Radial R;
  R.TB = (1.0 - J0e) * ir;
  R.TC0 = eps * J1e * ir;
  const double c20 = 2.0 * (1.0 - J0e) * ir * ir - eps * J1e * ir;
  R.TC2 = c20;
  const double d10 = eps * eps * J2e * ir;
  R.TD1 = d10;
  R.TD3 = 4.0 * ir * c20 - d10;
  R.TA = le * d10 - ir * c20;
  R.TL = le * R.TC0 - R.TB * ir;
  for (int q = 0; q < Qg; ++q) {
    const double r = rg[q], w = wyg[q], z = rho * r, lr = log(r);
    const double b0 = j0(z), b1 = j1(z), b2 = jn(2, z), b3 = jn(3, z);
    const double wr = w * r, wr2 = wr * r;
    R.TA = fma(wr2 * lr, b1, R.TA);
    R.TB = fma(w, b1, R.TB);
    R.TC0 = fma(wr, b0, R.TC0);
    R.TC2 = fma(wr, b2, R.TC2);
    R.TD1 = fma(wr2, b1, R.TD1);
    R.TD3 = fma(wr2, b3, R.TD3);
    R.TL = fma(wr * lr, b0, R.TL);
  }
  return R;
}

__global__ void k_sing2d_grad(int M1, int M2, double c_tilde, double A2, double eps, int Qg,
                              const double* __restrict__ rg, const double* __restrict__ wyg, double* __restrict__ D) {
  const long n = (long)M1 * M2;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int j1p = (int)(idx % M1), j2p = (int)(idx / M1);
  const double e1 = centered(j1p, M1), J = centered(j2p, M2) * kPi / c_tilde;
  const double rho = sqrt(e1 * e1 + J * J);
  double t[8];
  if (rho == 0.0) {
    // only the n = 0 term survives: Q1 = -(A2/2) int_0^{2eps} Y r dr
    double tc0 = 0.5 * eps * eps;
    for (int q = 0; q < Qg; ++q) tc0 = fma(wyg[q], rg[q], tc0);
#pragma unroll
    for (int m = 0; m < 8; ++m) t[m] = 0.0;
    t[2] = -0.5 * A2 * tc0;
  } else {
    const Radial R = radial_integrals(rho, eps, Qg, rg, wyg);
    const double cp = e1 / rho, sp = J / rho;
    const double c2p = cp * cp - sp * sp, s2p = 2.0 * sp * cp;
    const double c3p = cp * (4.0 * cp * cp - 3.0), s3p = sp * (3.0 - 4.0 * sp * sp);
    t[0] = -0.5 * A2 * cp * R.TA;
    t[1] = A2 * cp * R.TB;
    t[2] = -0.5 * A2 * (R.TC0 - c2p * R.TC2);
    t[3] = -0.25 * A2 * (c3p * R.TD3 - 3.0 * cp * R.TD1);
    t[4] = -0.5 * A2 * sp * R.TA;
    t[5] = A2 * sp * R.TB;
    t[6] = 0.5 * A2 * s2p * R.TC2;
    t[7] = -0.25 * A2 * (s3p * R.TD3 - sp * R.TD1);
  }
#pragma unroll
  for (int m = 0; m < 8; ++m) D[m * n + idx] = t[m];
}

// Tables of the second-derivative differences (Section 2.4.2): the singular parts
//   h11 = C (ln r/2 - i alpha x1 ln r/2 + x1^2/(2r^2) - i alpha x1^3/(2r^2)) Y,
//   h12 = C (x1 x2/(2r^2) - i alpha x1^2 x2/(2r^2)) Y,
//   h22 = C (ln r/2 - i alpha x1 ln r/2 + x2^2/(2r^2) - i alpha x1 x2^2/(2r^2)) Y,
// C = (k1^2 - k2^2)/(2 pi), have real coefficients H-hat_pq = C (u_pq + alpha v_pq) (the
// alpha-terms are odd in x1, so their transforms are imaginary and i alpha makes them real):
// six real tables u11 v11 u12 v12 u22 v22, [6][M2][M1], A2 and pi included.
__global__ void k_sing2d_hess(int M1, int M2, double c_tilde, double A2, double eps, int Qg,
                              const double* __restrict__ rg, const double* __restrict__ wyg, double* __restrict__ D) {
  const long n = (long)M1 * M2;
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= n) return;
  const int j1p = (int)(idx % M1), j2p = (int)(idx / M1);
  const double e1 = centered(j1p, M1), J = centered(j2p, M2) * kPi / c_tilde;
  const double rho = sqrt(e1 * e1 + J * J);
  const double s = A2 * kPi;
  double t[6];
  if (rho == 0.0) {
    // n = 0 terms only: TL(0) = int ln r Y r dr, TC0(0) = int Y r dr
    double tl = eps * eps * (0.5 * log(eps) - 0.25), tc0 = 0.5 * eps * eps;
    for (int q = 0; q < Qg; ++q) {
      tl = fma(wyg[q] * rg[q], log(rg[q]), tl);
      tc0 = fma(wyg[q], rg[q], tc0);
    }
#pragma unroll
    for (int m = 0; m < 6; ++m) t[m] = 0.0;
    t[0] = t[4] = s * (tl + 0.5 * tc0);
  } else {
    const Radial R = radial_integrals(rho, eps, Qg, rg, wyg);
    const double cp = e1 / rho, sp = J / rho;
    const double c2p = cp * cp - sp * sp, s2p = 2.0 * sp * cp;
    const double c3p = cp * (4.0 * cp * cp - 3.0), s3p = sp * (3.0 - 4.0 * sp * sp);
    t[0] = s * (R.TL + 0.5 * (R.TC0 - c2p * R.TC2));
    t[1] = s * (-cp * R.TA + 0.25 * (c3p * R.TD3 - 3.0 * cp * R.TD1));
    t[2] = s * (-0.5 * s2p * R.TC2);
    t[3] = s * (0.25 * (s3p * R.TD3 - sp * R.TD1));
    t[4] = s * (R.TL + 0.5 * (R.TC0 + c2p * R.TC2));
    t[5] = s * (-cp * R.TA - 0.25 * (cp * R.TD1 + c3p * R.TD3));
  }
#pragma unroll
  for (int m = 0; m < 6; ++m) D[m * n + idx] = t[m];
}

// 2D gradient fill (Section 2.4.1): the two fields
//   L-hat_1 = i(alpha + j1) K-hat - H-hat_1,  L-hat_2 = i j2 (pi/c~) K-hat - H-hat_2,
// K-hat of (2.1) as in the fill of G, H-hat_p from the gradient tables.
template <typename T, bool SPEC>
__global__ __launch_bounds__(256) void k_fill2d_grad(FillArgs A, const double* __restrict__ xq,
                                                     const double* __restrict__ wxq, const double2* __restrict__ cs,
                                                     const double* __restrict__ D, cplx<T>* __restrict__ out) {
  extern __shared__ double2 sa[];
  const int ip = threadIdx.x % TP, lane = threadIdx.x / TP;
  const int j1p0 = blockIdx.x * TP;
  const int j1p = j1p0 + ip;
  const int j1 = centered(min(j1p, A.M1 - 1), A.M1);
  const double a = A.a1 + j1;
  const double2 b = beta_of(A.k, fabs(a));
  const bool use_I = b.y * A.c < 41.5;
  if (__syncthreads_or(use_I && j1p < A.M1)) pencil_weights<2>(A, j1p0, 0, xq, wxq, sa);
  __syncthreads();
  if (j1p >= A.M1) return;
  const double2* ap = sa + ip;
  const double lead0 = a * a - A.k * A.k;
  const size_t n = (size_t)A.M1 * A.Mt;
  const double k2 = A.k * A.k, al = A.a1, ha2 = 0.5 * A.a1 * A.a1;
  auto put = [&](int jtp, double J, double2 K) {
    const size_t o = (size_t)jtp * A.M1 + j1p;
    // H-hat_p = i s_p
    const double s1 = k2 * D[o] + D[n + o] - al * D[2 * n + o] - ha2 * D[3 * n + o];
    const double s2 = k2 * D[4 * n + o] + D[5 * n + o] - al * D[6 * n + o] - ha2 * D[7 * n + o];
    // times the basis normalisation A2 (the grid sum)
    store_c<T>(out, o, cscale(mk(-a * K.y, a * K.x - s1), A.A));
    store_c<T>(out + A.fstride, o, cscale(mk(-J * K.y, J * K.x - s2), A.A));
  };
  for (int jtp = lane; jtp < A.Mt; jtp += TL) {
    const int jt = centered(jtp, A.Mt);
    const double J = jt * kPi / A.c_tilde;
    double2 term = mk(0.0, 0.0);
    if (use_I) term = xprime_term(ap, cs + (size_t)abs(jt) * A.Q, A.Q, jt < 0 ? -1.0 : 1.0, J, b);
    put(jtp, J, cscale(cadd(term, mk(1.0 / (lead0 + J * J), 0.0)), A.A));
  }
  if constexpr (SPEC) {
    int js[2];
    special_jts(b, A, js);
    for (int s = 0; s < 2; ++s) {
      if (js[s] < 0 || js[s] % TL != lane) continue;
      const double J = centered(js[s], A.Mt) * kPi / A.c_tilde;
      put(js[s], J, cscale(khat_direct(b.x, J, A, xq), A.A));
    }
  }
}

// H(rho) = rho^-1 int_eps^{2eps} e^{ikr} (2ik Y' + Y'') sin(rho r) dr (the radial
// form of the integral in eq. 3.5), tabulated on rho = (m - 4) hd, m in [0, hn).
__global__ __launch_bounds__(256) void k_htable(int hn, double hd, double k, int Q, const double* __restrict__ rq,
                                                const double* __restrict__ wrq, const double* __restrict__ y1q,
                                                const double* __restrict__ y2q, double2* __restrict__ htab) {
  // one 64-lane wave per table entry, lanes over quadrature nodes
  const int lane = threadIdx.x & 63;
  const int m = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (m >= hn) return;
  const double rho = fabs((m - 4) * hd);
  double2 acc = mk(0.0, 0.0);
  for (int q = lane; q < Q; q += 64) {
    const double r = rq[q];
    double s, c;
    sincos(k * r, &s, &c);
    const double2 g = cmul(mk(c, s), mk(y2q[q], 2.0 * k * y1q[q]));
    const double sn = rho > 0.0 ? sin(rho * r) / rho : r;
    acc = cadd(acc, cscale(g, wrq[q] * sn));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc.x += __shfl_xor(acc.x, off, 64);
    acc.y += __shfl_xor(acc.y, off, 64);
  }
  if (lane == 0) htab[m] = acc;
}

// Far slab, 3D (Algorithm 3.1 / 4.1 step 2b: the series (1.3)): per-slice coefficients
// (i/8pi^2) beta^-1 e^{i beta z_s} of the Mf1 x Mf2 lowest modes, z_s = z0 + s hf.  NFO = kMxO:
// the six entries of the Maxwell tensor (1.4) instead, the term times delta_pq - xi_p xi_q / k^2
// with xi = (alpha1 + j1, alpha2 + j2, beta) (the entries 13 and 23 take sgn(x3) at the target).

// i c beta^-1 e^{i beta z} (c real, z >= 0, beta from beta_of, so one of its parts is zero).  An
// evanescent mode (beta = i q) gives the real (c/q) e^{-qz}, a propagating one (beta = p)
// (c/p)(-sin pz, cos pz): one exponential or one sine-cosine pair, and one division.  The complex
// quotient and product written out in full take the same roundings, their other terms being exact
// zeros (up to the sign of a zero part); beta = 0, a Wood anomaly, is refused before any fill.
// Terms past the cut of far_negligible are taken as zero.
__device__ __forceinline__ double2 ibeta_exp(double c, double2 b, double z) {
  if (b.x == 0.0) {
    const double qz = b.y * z;
    return mk(qz > kFarNegligibleQz ? 0.0 : c / b.y * exp(-qz), 0.0);
  }
  double s, co;
  sincos(b.x * z, &s, &co);
  const double w = c / b.x;
  return mk(-(w * s), w * co);
}

// One far-slab coefficient of the series (1.3) in 3D: (i/8 pi^2) beta^-1 e^{i beta z} at mode
// (j1, j2) (FFT order) and height z.
__device__ __forceinline__ double2 far3_coef(double k, double a1, double a2, int M1, int M2, double z, int j1p,
                                             int j2p) {
  const double xi1 = a1 + centered(j1p, M1), xi2 = a2 + centered(j2p, M2);
  const double r2 = xi1 * xi1 + xi2 * xi2;
  if (far_negligible(r2, k, z)) return mk(0.0, 0.0);
  return ibeta_exp(1.0 / (8.0 * kPi * kPi), beta_of(k, sqrt(r2)), z);
}

// The Maxwell far slab's coefficients, one thread per (s, j2, j1) writing all six entries (beta and
// e^{i beta z} formed once for them); the x2 and x1 transforms follow as separate passes.
template <typename T>
__global__ void k_far3d_mx(double k, double a1, double a2, int M1, int M2, int S, double z0, double hf, long fstride,
                           cplx<T>* __restrict__ out) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M1 * M2 * S) return;
  const int j1p = (int)(idx % M1), j2p = (int)((idx / M1) % M2), s = (int)(idx / ((long)M1 * M2));
  const double xi1 = a1 + centered(j1p, M1), xi2 = a2 + centered(j2p, M2);
  const double r2 = xi1 * xi1 + xi2 * xi2, z = z0 + s * hf;
  if (far_negligible(r2, k, z)) {
#pragma unroll
    for (int f = 0; f < 6; ++f) store_c<T>(out, f * fstride + idx, mk(0.0, 0.0));
    return;
  }
  const double2 b = beta_of(k, sqrt(r2));
  const double2 v = ibeta_exp(1.0 / (8.0 * kPi * kPi), b, z);
  const double ik2 = 1.0 / (k * k);
  const double2 cc[3] = {mk(xi1, 0.0), mk(xi2, 0.0), b};
  const int P[6] = {0, 1, 2, 0, 0, 1}, Qp[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    const double2 m = cscale(cmul(cc[P[f]], cc[Qp[f]]), -ik2);
    store_c<T>(out, f * fstride + idx, cmul(v, mk((f < 3 ? 1.0 : 0.0) + m.x, m.y)));
  }
}

// The same six entries generated straight into LDS for `tile` rows (s, j2) of x1 coefficients,
// the inverse DFT along x1 run there on all 6 tile rows, and the rows written out (the x2
// transform follows as a column pass): one write of the slab instead of a write, then a read and
// a write by the x1 row pass.  LDS: [entry][row][j1'], then the twiddles when they fit.
template <typename T>
__global__ __launch_bounds__(256) void k_far3d_mx_rows(double k, double a1, double a2, int M1, int M2, int S,
                                                       double z0, double hf, int tile, long fstride,
                                                       const cplx<T>* __restrict__ tw, int ntw,
                                                       cplx<T>* __restrict__ out) {
  extern __shared__ char smem_raw[];
  using V = cplx<T>;
  const int n = M1;
  V* buf = reinterpret_cast<V*>(smem_raw);
  const long nrows = (long)M2 * S, r0 = (long)blockIdx.x * tile;
  const int ntile = (int)min((long)tile, nrows - r0);
  const double ik2 = 1.0 / (k * k);
  const int P[6] = {0, 1, 2, 0, 0, 1}, Qp[6] = {0, 1, 2, 1, 2, 2};
  // rows (s, j2) of far_band_empty are left unwritten: the x2 pass takes them as zero unread
  __shared__ unsigned char wr[64];
  if ((int)threadIdx.x < tile) {
    const int t = threadIdx.x;
    const long r = r0 + t;
    const int s = (int)(r / M2);
    wr[t] = t < ntile && !far_band_empty(a2 + centered((int)(r - (long)s * M2), M2), k, z0, hf, s);
  }
  bool nz = false;
  for (int idx = threadIdx.x; idx < tile * n; idx += blockDim.x) {
    const int t = idx / n, j1p = idx - t * n;
    if (t < ntile) {
      const long r = r0 + t;
      const int s = (int)(r / M2), j2p = (int)(r - (long)s * M2);
      const double xi1 = a1 + centered(j1p, M1), xi2 = a2 + centered(j2p, M2);
      const double r2 = xi1 * xi1 + xi2 * xi2, z = z0 + s * hf;
      if (far_negligible(r2, k, z)) {
#pragma unroll
        for (int f = 0; f < 6; ++f) store_c<T>(buf, (size_t)(f * tile + t) * n + j1p, mk(0.0, 0.0));
        continue;
      }
      nz = true;
      const double2 b = beta_of(k, sqrt(r2));
      const double2 v = ibeta_exp(1.0 / (8.0 * kPi * kPi), b, z);
      const double2 cc[3] = {mk(xi1, 0.0), mk(xi2, 0.0), b};
#pragma unroll
      for (int f = 0; f < 6; ++f) {
        const double2 m = cscale(cmul(cc[P[f]], cc[Qp[f]]), -ik2);
        store_c<T>(buf, (size_t)(f * tile + t) * n + j1p, cmul(v, mk((f < 3 ? 1.0 : 0.0) + m.x, m.y)));
      }
    }
  }
  // tiles whose every term is past the cut transform to zeros, written at once
  if (!__syncthreads_or(nz)) {
    V zero;
    zero.x = (T)0;
    zero.y = (T)0;
    for (int idx = threadIdx.x; idx < 6 * tile * n; idx += blockDim.x) {
      const int fr = idx / n, i1 = idx - fr * n, f = fr / tile, t = fr - f * tile;
      if (wr[t]) out[f * fstride + (r0 + t) * n + i1] = zero;
    }
    return;
  }
  // rows of the last block beyond the slab hold stale LDS: transformed, never written
  if (fft_twiddles_in_lds(6 * tile, n, n, sizeof(V))) {
    V* twl = buf + 6 * tile * n;
    const int stride = ntw / n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) twl[j] = tw[(long)j * stride];
    __syncthreads();
    fftdev::inverse_dft_lds<T>(buf, n, n, 6 * tile, twl, n);
  } else {
    fftdev::inverse_dft_lds<T>(buf, n, n, 6 * tile, tw, ntw);
  }
  for (int idx = threadIdx.x; idx < 6 * tile * n; idx += blockDim.x) {
    const int fr = idx / n, i1 = idx - fr * n, f = fr / tile, t = fr - f * tile;
    if (wr[t]) out[f * fstride + (r0 + t) * n + i1] = buf[idx];
  }
}

// The G_d far slab [s][i2][i1]: its coefficients are generated straight into LDS for a tile of
// adjacent x1 columns and the inverse DFT along x2 runs there (the first of its two transform
// passes; the coefficients never go to memory).  Batch b: slice b / M1, column b % M1.
template <typename T>
__global__ __launch_bounds__(256) void k_far3d_cols(double k, double a1, double a2, int M1, int M2, int S, double z0,
                                                    double hf, int tile, const cplx<T>* __restrict__ tw,
                                                    int ntw, cplx<T>* __restrict__ out) {
  extern __shared__ char smem_raw[];
  using V = cplx<T>;
  const int n = M2, pitch = n + 1;
  V* buf = reinterpret_cast<V*>(smem_raw);
  const long nbatch = (long)M1 * S;
  const long b0 = (long)blockIdx.x * tile;
  const int ntile = (int)min((long)tile, nbatch - b0);
  const int total = tile * n;
  // columns of far_band_empty are left unwritten: the x1 pass takes them as zero unread
  __shared__ unsigned char wr[64];
  if ((int)threadIdx.x < tile) {
    const int t = threadIdx.x;
    const long b = b0 + t;
    const long s = b / M1;
    wr[t] = t < ntile && !far_band_empty(a1 + centered((int)(b - s * M1), M1), k, z0, hf, s);
  }
  bool nz = false;
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int e = idx / tile, t = idx - e * tile;
    if (t < ntile) {
      const long b = b0 + t;
      const long s = b / M1;
      const int j1p = (int)(b - s * M1);
      const double2 v = far3_coef(k, a1, a2, M1, M2, z0 + s * hf, j1p, e);
      nz |= v.x != 0.0 || v.y != 0.0;
      V c;
      c.x = (T)v.x;
      c.y = (T)v.y;
      buf[t * pitch + e] = c;
    }
  }
  // tiles whose every term is past the cut transform to zeros, written at once
  if (!__syncthreads_or(nz)) {
    V zero;
    zero.x = (T)0;
    zero.y = (T)0;
    for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
      const int e = idx / tile, t = idx - e * tile;
      if (wr[t]) {
        const long b = b0 + t;
        const long plane = b / M1;
        out[plane * ((long)M1 * M2) + (long)e * M1 + (b - plane * M1)] = zero;
      }
    }
    return;
  }
  if (fft_twiddles_in_lds(tile, pitch, n, sizeof(V))) {
    V* twl = buf + tile * pitch;
    const int stride = ntw / n;
    for (int j = threadIdx.x; j < n; j += blockDim.x) twl[j] = tw[(long)j * stride];
    __syncthreads();
    fftdev::inverse_dft_lds<T>(buf, n, pitch, ntile, twl, n);
  } else {
    fftdev::inverse_dft_lds<T>(buf, n, pitch, ntile, tw, ntw);
  }
  for (int idx = threadIdx.x; idx < total; idx += blockDim.x) {
    const int e = idx / tile, t = idx - e * tile;
    if (wr[t]) {
      const long b = b0 + t;
      const long plane = b / M1;
      out[plane * ((long)M1 * M2) + (long)e * M1 + (b - plane * M1)] = buf[t * pitch + e];
    }
  }
}

// Fill of the second-derivative differences (Section 2.4.2): three fields
//   L-hat_pq = m_pq (K-hat^{(k1)} - K-hat^{(k2)}) - H-hat_pq,
// m_11 = -(alpha + j1)^2, m_12 = -(alpha + j1) J, m_22 = -J^2 (J = j2 pi/c~), K-hat of (2.1)
// for both wavenumbers (two sets of pencil weights in LDS); the difference of the leading
// terms 1/(|xi|^2 - k^2) is formed exactly as (k1^2 - k2^2)/((|xi|^2 - k1^2)(|xi|^2 - k2^2)).
template <typename T, bool SPEC>
__global__ __launch_bounds__(256) void k_fill2d_hess(FillArgs A, const double* __restrict__ xq,
                                                     const double* __restrict__ wxq, const double2* __restrict__ cs,
                                                     const double* __restrict__ D, cplx<T>* __restrict__ out) {
  extern __shared__ double2 sa[];
  const int ip = threadIdx.x % TP, lane = threadIdx.x / TP;
  const int j1p0 = blockIdx.x * TP;
  const int j1p = j1p0 + ip;
  const int j1 = centered(min(j1p, A.M1 - 1), A.M1);
  const double a = A.a1 + j1;
  FillArgs B = A;
  B.k = A.k2;
  const double2 b1 = beta_of(A.k, fabs(a)), b2 = beta_of(A.k2, fabs(a));
  const bool use1 = b1.y * A.c < 41.5, use2 = b2.y * A.c < 41.5;
  double2* sa2 = sa + TP * A.Q;
  if (__syncthreads_or(use1 && j1p < A.M1)) pencil_weights<2>(A, j1p0, 0, xq, wxq, sa);
  if (__syncthreads_or(use2 && j1p < A.M1)) pencil_weights<2>(B, j1p0, 0, xq, wxq, sa2);
  __syncthreads();
  if (j1p >= A.M1) return;
  const size_t n = (size_t)A.M1 * A.Mt;
  const double k1s = A.k * A.k, k2s = A.k2 * A.k2;
  const double C = (k1s - k2s) / (2.0 * kPi);
  auto put = [&](int jtp, double J, double2 dK) {
    dK = cscale(dK, A.A);
    const size_t o = (size_t)jtp * A.M1 + j1p;
    const double h11 = C * (D[o] + A.a1 * D[n + o]);
    const double h12 = C * (D[2 * n + o] + A.a1 * D[3 * n + o]);
    const double h22 = C * (D[4 * n + o] + A.a1 * D[5 * n + o]);
    store_c<T>(out, o, cscale(mk(-a * a * dK.x - h11, -a * a * dK.y), A.A));
    store_c<T>(out + A.fstride, o, cscale(mk(-a * J * dK.x - h12, -a * J * dK.y), A.A));
    store_c<T>(out + 2 * A.fstride, o, cscale(mk(-J * J * dK.x - h22, -J * J * dK.y), A.A));
  };
  for (int jtp = lane; jtp < A.Mt; jtp += TL) {
    const int jt = centered(jtp, A.Mt);
    const double J = jt * kPi / A.c_tilde;
    const double d = a * a + J * J;
    const double sg = jt < 0 ? -1.0 : 1.0;
    double2 dK = mk((k1s - k2s) / ((d - k1s) * (d - k2s)), 0.0);
    if (use1) dK = cadd(dK, xprime_term(sa + ip, cs + (size_t)abs(jt) * A.Q, A.Q, sg, J, b1));
    if (use2) dK = csub(dK, xprime_term(sa2 + ip, cs + (size_t)abs(jt) * A.Q, A.Q, sg, J, b2));
    put(jtp, J, dK);
  }
  if constexpr (SPEC) {
    // a special coefficient of either wavenumber: the two K-hat separately, the special
    // one(s) from the defining integral
    int js[4];
    special_jts(b1, A, js);
    special_jts(b2, A, js + 2);
    for (int s = 0; s < 4; ++s) {
      const int jtp = js[s];
      if (jtp < 0 || jtp % TL != lane || (s >= 2 && (jtp == js[0] || jtp == js[1]))) continue;
      const int jt = centered(jtp, A.Mt);
      const double J = jt * kPi / A.c_tilde;
      const double d = a * a + J * J;
      const double sg = jt < 0 ? -1.0 : 1.0;
      const bool s1 = jtp == js[0] || jtp == js[1], s2 = jtp == js[2] || jtp == js[3];
      double2 K1, K2;
      if (s1) {
        K1 = khat_direct(b1.x, J, A, xq);
      } else {
        K1 = mk(1.0 / (d - k1s), 0.0);
        if (use1) K1 = cadd(K1, xprime_term(sa + ip, cs + (size_t)abs(jt) * A.Q, A.Q, sg, J, b1));
      }
      if (s2) {
        K2 = khat_direct(b2.x, J, A, xq);
      } else {
        K2 = mk(1.0 / (d - k2s), 0.0);
        if (use2) K2 = cadd(K2, xprime_term(sa2 + ip, cs + (size_t)abs(jt) * A.Q, A.Q, sg, J, b2));
      }
      put(jtp, J, csub(K1, K2));
    }
  }
}

// Far slab, 2D (Algorithm 2.1 step 2b: the series (1.2)): (i/4pi) beta_n^-1 e^{i beta_n z_s} of the
// M1 lowest modes, z_s = z0 + s hf.
template <typename T>
__global__ void k_far2d(double k, double a, int M1, int S, double z0, double hf, cplx<T>* __restrict__ out) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M1 * S) return;
  const int j1p = (int)(idx % M1), s = (int)(idx / M1);
  const double2 b = beta_of(k, fabs(a + centered(j1p, M1)));
  const double z = z0 + s * hf;
  store_c<T>(out, idx, ibeta_exp(1.0 / (4.0 * kPi), b, z));
}

// Far slab of the 2D gradient: the coefficients of the series (1.2) differentiated,
// i(alpha + n) (i/4pi) beta_n^-1 e^{i beta_n z_s} for x1 and i beta_n (i/4pi) beta_n^-1 e^{i beta_n z_s}
// = -(1/4pi) e^{i beta_n z_s} for x2 (the factor sgn(x2) is applied at the target).
template <typename T>
__global__ void k_far2d_grad(double k, double a, int M1, int S, double z0, double hf, long fstride,
                             cplx<T>* __restrict__ out) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M1 * S) return;
  const int j1p = (int)(idx % M1), s = (int)(idx / M1);
  const double an = a + centered(j1p, M1);
  const double2 b = beta_of(k, fabs(an));
  const double2 e = cexpi(cscale(b, z0 + s * hf));
  const double2 f = cmul(cdiv(mk(0.0, 1.0 / (4.0 * kPi)), b), e);
  store_c<T>(out, idx, mk(-an * f.y, an * f.x));
  store_c<T>(out + fstride, idx, cscale(e, -1.0 / (4.0 * kPi)));
}

// Far slab of the second-derivative differences: the coefficients of (1.2) times -alpha_n^2,
// -alpha_n beta_n (sgn(x2) at the target) and -beta_n^2, for k1 minus for k2.
template <typename T>
__global__ void k_far2d_hess(double k1, double k2, double a, int M1, int S, double z0, double hf, long fstride,
                             cplx<T>* __restrict__ out) {
  const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)M1 * S) return;
  const int j1p = (int)(idx % M1), s = (int)(idx / M1);
  const double an = a + centered(j1p, M1), z = z0 + s * hf;
  double2 f11 = mk(0.0, 0.0), f12 = mk(0.0, 0.0), f22 = mk(0.0, 0.0);
  for (int w = 0; w < 2; ++w) {
    const double k = w == 0 ? k1 : k2, sg = w == 0 ? 1.0 : -1.0;
    const double2 b = beta_of(k, fabs(an));
    const double2 f = cscale(cmul(cdiv(mk(0.0, 1.0 / (4.0 * kPi)), b), cexpi(cscale(b, z))), sg);
    f11 = cadd(f11, cscale(f, -an * an));
    f12 = csub(f12, cscale(cmul(b, f), an));
    f22 = csub(f22, cmul(cmul(b, b), f));
  }
  store_c<T>(out, idx, f11);
  store_c<T>(out + fstride, idx, f12);
  store_c<T>(out + 2 * fstride, idx, f22);
}

// Far slab of many 2D instances: instance i owns blocks [blk0_i, blk0_{i+1}) of 256 threads.
template <typename T>
__global__ void k_far2d_multi(const FillInst* __restrict__ inst, int n_inst, cplx<T>* __restrict__ base) {
  const int i = find_inst(inst, n_inst, blockIdx.x);
  const FillInst I = inst[i];
  const long idx = (blockIdx.x - I.blk0) * (long)blockDim.x + threadIdx.x;
  if (idx >= (long)I.Mf1 * I.Sf) return;
  const int j1p = (int)(idx % I.Mf1), s = (int)(idx / I.Mf1);
  const double2 b = beta_of(I.A.k, fabs(I.A.a1 + centered(j1p, I.Mf1)));
  const double z = I.z0 + s * I.hf;
  store_c<T>(base + I.foff, idx, ibeta_exp(1.0 / (4.0 * kPi), b, z));
}

template <typename T>
hipError_t fill_impl(Plan& P, double k, double a1, double a2, bool fuse, bool spec) {
  FillArgs A;
  A.k = k;
  A.a1 = a1;
  A.a2 = a2;
  A.c = P.p.c;
  A.c_tilde = P.p.c_tilde;
  A.M1 = P.M1;
  A.M2 = P.M2;
  A.Mt = P.Mt;
  A.Q = P.p.quad_q;
  A.hd = P.hd;
  A.fstride = (long)P.ncell;
  A.stol = P.p.special_tol;
  A.wXq = P.wXq;
  A.rq = P.rq;
  A.wrq = P.wrq;
  A.Qr = P.Qr;
  A.eps = P.p.eps;
  A.E = P.E2;
  A.sing_order = P.p.sing_order;
  const size_t shm = (size_t)TP * A.Q * sizeof(double2);
  auto* out = static_cast<cplx<T>*>(P.grid);
  if (P.dim == 2) {
    A.A = 1.0 / (2.0 * sqrt(kPi * A.c_tilde));
    dim3 grid((P.M1 + TP - 1) / TP, 1);
    A.k2 = P.last_k2;
    // the special-coefficient path is compiled in only for instances that have one
    if (P.nf == 2) {
      if (spec)
        hipLaunchKernelGGL((k_fill2d_grad<T, true>), grid, dim3(TP * TL), shm, P.stream, A, P.xq, P.wxq, P.cs, P.D2,
                           out);
      else
        hipLaunchKernelGGL((k_fill2d_grad<T, false>), grid, dim3(TP * TL), shm, P.stream, A, P.xq, P.wxq, P.cs,
                           P.D2, out);
    } else if (P.nf == 3) {
      if (spec)
        hipLaunchKernelGGL((k_fill2d_hess<T, true>), grid, dim3(TP * TL), 2 * shm, P.stream, A, P.xq, P.wxq, P.cs,
                           P.D2, out);
      else
        hipLaunchKernelGGL((k_fill2d_hess<T, false>), grid, dim3(TP * TL), 2 * shm, P.stream, A, P.xq, P.wxq, P.cs,
                           P.D2, out);
    } else {
      if (spec)
        hipLaunchKernelGGL((k_fill2d<T, true>), grid, dim3(TP * TL), shm, P.stream, A, P.xq, P.wxq, P.cs, P.F1, P.F2,
                           out);
      else
        hipLaunchKernelGGL((k_fill2d<T, false>), grid, dim3(TP * TL), shm, P.stream, A, P.xq, P.wxq, P.cs, P.F1,
                           P.F2, out);
    }
  } else {
    A.A = 1.0 / sqrt(8.0 * kPi * kPi * A.c_tilde);
    dim3 grid((P.M1 + TP - 1) / TP, P.M2);
    const cplx<T>* tw = nullptr;
    if constexpr (sizeof(T) == 8) tw = P.tw; else tw = P.twf;
    const size_t shf = shm + (size_t)P.nf * TP * (P.Mt + 1) * sizeof(cplx<T>);
#define QPGF_FILL3D(NF_, FUSE_, SHM_)                                                                              \
  do {                                                                                                              \
    if (spec)                                                                                                       \
      hipLaunchKernelGGL((k_fill3d<T, NF_, FUSE_, true>), grid, dim3(TP * TL), SHM_, P.stream, A, P.xq, P.wxq, P.cs, \
                         P.htab, out, tw, P.ntw);                                                                   \
    else                                                                                                            \
      hipLaunchKernelGGL((k_fill3d<T, NF_, FUSE_, false>), grid, dim3(TP * TL), SHM_, P.stream, A, P.xq, P.wxq,      \
                         P.cs, P.htab, out, tw, P.ntw);                                                             \
  } while (0)
    if (P.nf == kMxF) {
      if (fuse) QPGF_FILL3D(kMxF, true, shf);
      else QPGF_FILL3D(kMxF, false, shm);
    } else if (P.nf == kMxT) {
      if (fuse) QPGF_FILL3D(kMxT, true, shf);
      else QPGF_FILL3D(kMxT, false, shm);
    } else if (fuse) {
      QPGF_FILL3D(1, true, shf);
    } else {
      QPGF_FILL3D(1, false, shm);
    }
#undef QPGF_FILL3D
  }
  return hipGetLastError();
}

template <typename T>
hipError_t far_impl(Plan& P, double k, double a1, double a2) {
  auto* out = static_cast<cplx<T>*>(P.far);
  const double hf = P.hf, z0 = P.fz0;
  const long n = (long)P.Mf1 * P.Mf2 * P.S;
  const dim3 g((unsigned)((n + 255) / 256)), b(256);
  if (P.dim == 2) {
    if (P.nf == 2)
      hipLaunchKernelGGL(k_far2d_grad<T>, g, b, 0, P.stream, k, a1, P.Mf1, P.S, z0, hf, (long)P.nfar, out);
    else if (P.nf == 3)
      hipLaunchKernelGGL(k_far2d_hess<T>, g, b, 0, P.stream, k, P.last_k2, a1, P.Mf1, P.S, z0, hf, (long)P.nfar, out);
    else
      hipLaunchKernelGGL(k_far2d<T>, g, b, 0, P.stream, k, a1, P.Mf1, P.S, z0, hf, out);
  } else if (P.nfo == kMxO && far_rows_in_fill(P)) {
    // coefficients and the x1 transform in one pass (the x2 pass follows in the caller)
    const int n = P.Mf1, tile = std::max(1, std::min(fftdev::lds_cap<T>() / (6 * n), 4));
    const size_t shm = ((size_t)6 * tile * n + (fft_twiddles_in_lds(6 * tile, n, n, sizeof(cplx<T>)) ? n : 0)) *
                       sizeof(cplx<T>);
    const cplx<T>* tw = nullptr;
    if constexpr (sizeof(T) == 8) tw = P.tw; else tw = P.twf;
    const long nrows = (long)P.Mf2 * P.S;
    hipLaunchKernelGGL(k_far3d_mx_rows<T>, dim3((unsigned)((nrows + tile - 1) / tile)), dim3(256), shm, P.stream, k,
                       a1, a2, P.Mf1, P.Mf2, P.S, z0, hf, tile, (long)P.nfar, tw, P.ntw, out);
  } else if (P.nfo == kMxO) {
    hipLaunchKernelGGL(k_far3d_mx<T>, g, b, 0, P.stream, k, a1, a2, P.Mf1, P.Mf2, P.S, z0, hf, (long)P.nfar, out);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_fft(P, P.far, P.Mf2, P.Mf1, (long)P.Mf1 * P.S * P.nfo, P.Mf1, 1, (long)P.Mf1 * P.Mf2);
  } else {
    // coefficients and the x2 transform in one pass (the x1 pass follows in the caller)
    const int n = P.Mf2, pitch = n + 1;
    const long nbatch = (long)P.Mf1 * P.S;
    const int tile = std::min(fft_tile(P, n, false, nbatch), 64);   // the kernel's column flags hold 64
    const size_t shm = ((size_t)tile * pitch + (fft_twiddles_in_lds(tile, pitch, n, sizeof(cplx<T>)) ? n : 0)) *
                       sizeof(cplx<T>);
    const cplx<T>* tw = nullptr;
    if constexpr (sizeof(T) == 8) tw = P.tw; else tw = P.twf;
    const dim3 gb((unsigned)((nbatch + tile - 1) / tile));
    hipLaunchKernelGGL(k_far3d_cols<T>, gb, dim3(256), shm, P.stream, k, a1, a2, P.Mf1, P.Mf2, P.S, z0, hf,
                       tile, tw, P.ntw, out);
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_sing2d(Plan& P, double f1zero) {
  const long n = (long)P.M1 * P.M2;
  const double A2 = 1.0 / (2.0 * sqrt(kPi * P.p.c_tilde));
  hipLaunchKernelGGL(k_sing2d, dim3((n + 255) / 256), dim3(256), 0, P.stream, P.M1, P.M2, P.p.c_tilde, A2,
                     P.Qr, P.rq, P.wrq, f1zero, P.F1, P.F2);
  return hipGetLastError();
}

hipError_t launch_sing2d_ho(Plan& P, int Qg, const double* rg, const double* wyg) {
  const long n = (long)P.M1 * P.M2;
  const double A2 = 1.0 / (2.0 * sqrt(kPi * P.p.c_tilde));
  hipLaunchKernelGGL(k_sing2d_ho, dim3((n + 255) / 256), dim3(256), 0, P.stream, P.M1, P.M2, P.p.c_tilde, A2,
                     P.p.eps, Qg, rg, wyg, P.E2);
  return hipGetLastError();
}

hipError_t launch_sing2d_grad(Plan& P, int Qg, const double* rg, const double* wyg) {
  const long n = (long)P.M1 * P.M2;
  const double A2 = 1.0 / (2.0 * sqrt(kPi * P.p.c_tilde));
  hipLaunchKernelGGL(k_sing2d_grad, dim3((n + 255) / 256), dim3(256), 0, P.stream, P.M1, P.M2, P.p.c_tilde, A2,
                     P.p.eps, Qg, rg, wyg, P.D2);
  return hipGetLastError();
}

hipError_t launch_sing2d_hess(Plan& P, int Qg, const double* rg, const double* wyg) {
  const long n = (long)P.M1 * P.M2;
  const double A2 = 1.0 / (2.0 * sqrt(kPi * P.p.c_tilde));
  hipLaunchKernelGGL(k_sing2d_hess, dim3((n + 255) / 256), dim3(256), 0, P.stream, P.M1, P.M2, P.p.c_tilde, A2,
                     P.p.eps, Qg, rg, wyg, P.D2);
  return hipGetLastError();
}

hipError_t launch_htable(Plan& P, double k) {
  hipLaunchKernelGGL(k_htable, dim3((P.hn + 3) / 4), dim3(256), 0, P.stream, P.hn, P.hd, k, P.Qr, P.rq,
                     P.wrq, P.y1q, P.y2q, P.htab);
  return hipGetLastError();
}

// host-side descriptor of one 2D instance for the batched launches
void fill_inst_2d(const Plan& P, double k, double a, int M1, const FarGeom& fg, long off, long foff, long blk0,
                  void* dst) {
  FillInst I;
  I.A.k = k;
  I.A.a1 = a;
  I.A.a2 = 0.0;
  I.A.c = P.p.c;
  I.A.c_tilde = P.p.c_tilde;
  I.A.A = 1.0 / (2.0 * sqrt(kPi * P.p.c_tilde));
  I.A.M1 = M1;
  I.A.M2 = P.M2;
  I.A.Mt = P.M2;
  I.A.Q = P.p.quad_q;
  I.A.hd = P.hd;
  I.A.fstride = (long)M1 * P.M2;
  I.A.stol = P.p.special_tol;
  I.A.wXq = P.wXq;
  I.A.rq = P.rq;
  I.A.wrq = P.wrq;
  I.A.Qr = P.Qr;
  I.A.eps = P.p.eps;
  I.A.k2 = 0.0;
  I.A.E = P.E2;
  I.A.sing_order = P.p.sing_order;
  I.Mf1 = fg.Mf1;
  I.Sf = fg.S;
  I.hf = fg.hf;
  I.z0 = P.p.c - (fg.P / 2 - 1) * fg.hf;
  I.off = off;
  I.foff = foff;
  I.blk0 = blk0;
  *static_cast<FillInst*>(dst) = I;
}
size_t fill_inst_size() { return sizeof(FillInst); }

hipError_t launch_fill2d_multi(Plan& P, const void* dinst, int n_inst, long nblocks, void* base, bool spec) {
  const size_t shm = (size_t)TP * P.p.quad_q * sizeof(double2);
  const auto* in = static_cast<const FillInst*>(dinst);
  const dim3 g((unsigned)nblocks), b(TP * TL);
  if (P.p.prec == QPGF_C128) {
    auto* o = static_cast<double2*>(base);
    if (spec)
      hipLaunchKernelGGL((k_fill2d_multi<double, true>), g, b, shm, P.stream, in, n_inst, P.xq, P.wxq, P.cs, P.F1,
                         P.F2, P.M1, o);
    else
      hipLaunchKernelGGL((k_fill2d_multi<double, false>), g, b, shm, P.stream, in, n_inst, P.xq, P.wxq, P.cs, P.F1,
                         P.F2, P.M1, o);
  } else {
    auto* o = static_cast<float2*>(base);
    if (spec)
      hipLaunchKernelGGL((k_fill2d_multi<float, true>), g, b, shm, P.stream, in, n_inst, P.xq, P.wxq, P.cs, P.F1,
                         P.F2, P.M1, o);
    else
      hipLaunchKernelGGL((k_fill2d_multi<float, false>), g, b, shm, P.stream, in, n_inst, P.xq, P.wxq, P.cs, P.F1,
                         P.F2, P.M1, o);
  }
  return hipGetLastError();
}

hipError_t launch_far2d_multi(Plan& P, const void* dinst, int n_inst, long nblocks, void* base) {
  const auto* in = static_cast<const FillInst*>(dinst);
  if (P.p.prec == QPGF_C128)
    hipLaunchKernelGGL(k_far2d_multi<double>, dim3((unsigned)nblocks), dim3(256), 0, P.stream, in, n_inst,
                       static_cast<double2*>(base));
  else
    hipLaunchKernelGGL(k_far2d_multi<float>, dim3((unsigned)nblocks), dim3(256), 0, P.stream, in, n_inst,
                       static_cast<float2*>(base));
  return hipGetLastError();
}

// The 3D fill takes the transverse transform over when the TP pencils of all its fields and the
// pencil weights fit together in 64 KiB of LDS (G_d up to long transverse axes; the Maxwell
// fields at complex64 with up to 32 slices).
bool fill_fuses_transverse(const Plan& P) {
  const size_t lds = (size_t)TP * P.p.quad_q * sizeof(double2) + (size_t)P.nf * TP * (P.Mt + 1) * P.esize;
  return P.dim == 3 && P.Mt > 1 && lds <= 65536;
}

hipError_t launch_fill(Plan& P, double k, double a1, double a2, bool fuse) {
  fuse = fuse && fill_fuses_transverse(P);
  const bool spec = P.spec;
  return P.p.prec == QPGF_C128 ? fill_impl<double>(P, k, a1, a2, fuse, spec)
                               : fill_impl<float>(P, k, a1, a2, fuse, spec);
}

// The Maxwell far slab's six entries of an x1 row (6 Mf1 values) fit one block's LDS: the far
// fill then runs the x1 transform, and the caller's second pass is the x2 columns.
bool far_rows_in_fill(const Plan& P) {
  return P.dim == 3 && P.nfo == kMxO && 6L * P.Mf1 * (long)P.esize <= 65536 - (long)P.Mf1 * (long)P.esize;
}

hipError_t launch_far(Plan& P, double k, double a1, double a2) {
  return P.p.prec == QPGF_C128 ? far_impl<double>(P, k, a1, a2) : far_impl<float>(P, k, a1, a2);
}

}  // namespace qpgf
