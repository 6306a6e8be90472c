// C ABI of libqpgf (include/qpgf.h): parameter validation, plan set-up
// (quadrature rules, twiddles, the 2D singular tables of Remark 2.1), the
// host-side exclusion checks (Wood anomalies, Section 1; the special
// coefficients of Sections 2.1 / 3.1) and the preparation / calculation
// sequences of Algorithms 2.1, 3.1 and 4.1.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "fft_device.h"
#include "qpgf_internal.h"

using namespace qpgf;

struct qpgf_plan {
  Plan P;
};

namespace {

thread_local std::string g_err;
constexpr long double kPiL = 3.141592653589793238462643383279502884L;

qpgf_status fail(qpgf_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

qpgf_status hip_fail(hipError_t e, const char* where) {
  return fail(e == hipErrorOutOfMemory ? QPGF_E_NOMEM : QPGF_E_HIP,
              std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) return hip_fail(e_, #call);  \
  } while (0)

bool pow2_in(int m, int lo, int hi) { return m >= lo && m <= hi && (m & (m - 1)) == 0; }
// x1 sizes of the 2D grids: m = 2^a r, a >= 1, r in {1, 3, 5, 7} (the transforms' radices)
bool m1_2d_in(int m, int lo, int hi) { return m >= lo && m <= hi && (m & 1) == 0 && fftdev::fft_length_ok(m); }

// Gauss-Legendre nodes and weights on [-1, 1] by Newton's method on P_n.
void gauss_legendre(int n, std::vector<long double>& x, std::vector<long double>& w) {
  x.assign(n, 0.0L);
  w.assign(n, 0.0L);
  for (int i = 0; i < n; ++i) {
    long double z = cosl(kPiL * (i + 0.75L) / (n + 0.5L));
    long double dp = 0.0L;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1.0L, p1 = z;
      for (int m = 2; m <= n; ++m) {
        long double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
      long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    {
      long double p0 = 1.0L, p1 = z;
      for (int m = 2; m <= n; ++m) {
        long double p2 = ((2 * m - 1) * z * p1 - (m - 1) * p0) / m;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0L);
    }
    x[i] = -z;
    w[i] = 2.0L / ((1.0L - z * z) * dp * dp);
  }
}

template <typename V>
qpgf_status upload(V** dst, const std::vector<V>& src) {
  HIP_TRY(hipMalloc(reinterpret_cast<void**>(dst), src.size() * sizeof(V)));
  HIP_TRY(hipMemcpy(*dst, src.data(), src.size() * sizeof(V), hipMemcpyHostToDevice));
  return QPGF_OK;
}

void free_batch(Plan& P) {
  if (P.b_exec) (void)hipGraphExecDestroy(P.b_exec);
  if (P.b_graph) (void)hipGraphDestroy(P.b_graph);
  P.b_exec = nullptr;
  P.b_graph = nullptr;
  P.b_sig.clear();
}

void free_plan(Plan& P) {
  free_batch(P);
  if (P.ws) {   // the caller's memory
    P.grid = P.far = P.gridI = P.farI = nullptr;
  }
  if (P.side) (void)hipStreamDestroy(P.side);
  if (P.ev_fork) (void)hipEventDestroy(P.ev_fork);
  if (P.ev_join) (void)hipEventDestroy(P.ev_join);
  if (P.b_capture) (void)hipStreamDestroy(P.b_capture);
  if (P.b_upload_done) (void)hipEventDestroy(P.b_upload_done);
  if (P.b_host) (void)hipHostFree(P.b_host);
  for (void* q : {P.b_grid, P.b_far, P.b_desc, P.gridI})
    if (q) (void)hipFree(q);
  free_target_scratch(P.ts);
  void* ptrs[] = {P.grid, P.far, P.farI, P.xq, P.wxq, P.wXq, P.cs, P.rq, P.wrq, P.y1q, P.y2q, P.tw, P.twf, P.F1, P.F2,
                  P.D2, P.E2, P.htab};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

bool kind_is_2d(int kind) {
  return kind == QPGF_KIND_G2D || kind == QPGF_KIND_G2D_GRAD || kind == QPGF_KIND_G2D_HESS_DIFF;
}

qpgf_status validate(const qpgf_params* p) {
  if (!p) return fail(QPGF_E_ARG, "params is NULL");
  if (p->kind < 0 || p->kind > 4) return fail(QPGF_E_ARG, "unknown kind");
  if (p->prec != QPGF_C128 && p->prec != QPGF_C64) return fail(QPGF_E_ARG, "unknown precision");
  if (kind_is_2d(p->kind) ? !m1_2d_in(p->m1, 16, 4096) : !pow2_in(p->m1, 16, 4096))
    return fail(QPGF_E_SIZE, "m1 must be in [16, 4096]: a power of two, or in 2D 2^a r with a >= 1 and r = 3, 5 or 7");
  if (!pow2_in(p->m2, 16, 4096)) return fail(QPGF_E_SIZE, "m2 must be a power of two in [16, 4096]");
  if (!kind_is_2d(p->kind) && !pow2_in(p->m3, 16, 4096))
    return fail(QPGF_E_SIZE, "m3 must be a power of two in [16, 4096]");
  {
    // one transform (padded for column axes) must fit the 64 KiB LDS buffer of a block
    const int lim = p->prec == QPGF_C128 ? 4096 : 8192;
    const bool bad = p->m1 > lim || p->m2 > lim / 2 || (!kind_is_2d(p->kind) && p->m3 > lim / 2);
    if (bad)
      return fail(QPGF_E_SIZE, "m1 <= 4096; complex128 column axes (m2, and m3 in 3D) <= 2048");
  }
  if (!(p->c > 0.0) || !(p->c_tilde > p->c)) return fail(QPGF_E_ARG, "need 0 < c < c_tilde");
  if (!(p->eps > 0.0) || !(2.0 * p->eps <= p->c_tilde)) return fail(QPGF_E_ARG, "need 0 < 2 eps <= c_tilde");
  if (p->quad_q < 16 || p->quad_q > 256) return fail(QPGF_E_ARG, "quad_q must be in [16, 256]");
  if (p->kind == QPGF_KIND_G2D_HESS_DIFF && p->quad_q > 128)
    return fail(QPGF_E_ARG, "quad_q must be <= 128 for QPGF_KIND_G2D_HESS_DIFF (two wavenumbers' weights in LDS)");
  if (!(p->far_h >= 0.0) || !(p->far_zmax >= p->c)) return fail(QPGF_E_ARG, "need far_h >= 0 and far_zmax >= c");
  if (p->far_h > 0.0 && (p->far_zmax - p->c) / p->far_h > 65536.0) return fail(QPGF_E_ARG, "far_h too small");
  if (!(p->wood_tol >= 0.0) || !(p->special_tol >= 0.0) || !(p->lattice_rmin >= 0.0))
    return fail(QPGF_E_ARG, "tolerances must be >= 0");
  if (!(p->special_tol < 0.25 * M_PI / p->c_tilde))
    return fail(QPGF_E_ARG, "special_tol must be below pi / (4 c_tilde)");
  if (p->sing_order < 1 || p->sing_order > 3) return fail(QPGF_E_ARG, "sing_order must be 1, 2 or 3");
  if (p->sing_order != 1 && p->kind != QPGF_KIND_G2D) return fail(QPGF_E_ARG, "sing_order above 1 needs QPGF_KIND_G2D");
  if (p->ring_interp != 0 && p->ring_interp != 1) return fail(QPGF_E_ARG, "ring_interp must be 0 or 1");
  if (p->ring_interp && p->kind != QPGF_KIND_G2D && p->kind != QPGF_KIND_G2D_GRAD && p->kind != QPGF_KIND_G2D_HESS_DIFF)
    return fail(QPGF_E_ARG, "ring_interp needs a 2D kind");
  if (p->far_m != 0) {
    if (!pow2_in(p->far_m, 16, 4096)) return fail(QPGF_E_SIZE, "far_m must be 0 or a power of two in [16, 4096]");
    if (!kind_is_2d(p->kind) && p->prec == QPGF_C128 && p->far_m > 2048)
      return fail(QPGF_E_SIZE, "complex128 3D plans: far_m <= 2048 (its x2 axis is transformed as columns)");
  }
  if (p->maxwell_trace != 0 && p->maxwell_trace != 1) return fail(QPGF_E_ARG, "maxwell_trace must be 0 or 1");
  if (p->maxwell_trace && p->kind != QPGF_KIND_MAXWELL3D) return fail(QPGF_E_ARG, "maxwell_trace needs QPGF_KIND_MAXWELL3D");
  return QPGF_OK;
}

}  // namespace

// Far-slab geometry (Algorithm 2.1 / 3.1 / 4.1 step 2b: the series on the slab, interpolated with
// the P-point Lagrange rule per axis).  The rule's error for a term of wavenumber q along an axis of
// spacing h is about C_P (q h)^P, C_8 = 1e-3, C_4 = 0.023: with h = 2 pi / Mf and the propagating terms
// (q <= k), Mf >= 2 pi k / x keeps it near 1e-11 for complex128 (P = 8, x = 0.0977) and 1e-6 for
// complex64 (P = 4, x = 0.081: 16 nodes per target in 2D and 64 in 3D instead of 64 and 512); the
// slice spacing follows the same rule with its own x.  The
// evanescent terms the series keeps just below c set the floors: hf <= 1/64, and 512 modes
// (complex128; 256 leave up to 4e-11 of |G_d| next to |x3| = c at k = 3.7, 512 leave 6e-13), 512 for
// complex64 in 3D, 256 for complex64 in 2D (3e-7 of the terms' size).  Slices z_s = c - (P/2 - 1) hf
// + s hf, s < S: a target at |x_t| = z uses slices floor((z - z_0) / hf) - (P/2 - 1) .. + P/2, so
// S = ceil((zmax - c) / hf) + P covers every z <= zmax.  params.far_m and params.far_h override the
// modes and the spacing.
FarGeom qpgf::far_geometry(const Plan& P, double kmax, int M1) {
  const bool c128 = P.p.prec == QPGF_C128;
  FarGeom g;
  g.P = c128 ? 8 : 4;
  const double x = c128 ? 0.0977 : 0.081;
  const int floor_m = (c128 || P.dim == 3) ? 512 : 256;
  const double want = 2.0 * M_PI * std::max(kmax, 0.0) / x;
  int mk = floor_m;
  while (mk < want && mk < 4096) mk <<= 1;
  const int cap = (P.dim == 3 && c128) ? 2048 : 4096;   // the 3D far slab's x2 axis is a column axis
  // at least the near grid's modes along x1, rounded up to a power of two (2D x1 sizes 2^a r)
  int m1f = 16;
  while (m1f < M1) m1f <<= 1;
  g.Mf1 = P.p.far_m ? P.p.far_m : std::min(std::max(m1f, mk), 4096);
  g.Mf2 = P.dim == 3 ? (P.p.far_m ? P.p.far_m : std::min(std::max(P.M2, mk), cap)) : 1;
  if (P.p.far_h > 0.0) {
    g.hf = P.p.far_h;
  } else {
    // the slice spacing: k hf <= 0.107 (complex128, 8 points: 1e-11) or 0.11 (complex64, 4 points:
    // 3e-6 of the series, against the complex64 bar of 1e-5)
    double inv = 64.0;
    const double need = std::max(kmax, 0.0) / (c128 ? 0.107 : 0.11);
    while (inv < need && inv < 4096.0) inv *= 2.0;
    g.hf = 1.0 / inv;
  }
  g.S = (int)std::ceil((P.p.far_zmax - P.p.c) / g.hf - 1e-12) + g.P;
  return g;
}

namespace {

// Take the far-slab geometry of an instance with largest wavenumber kmax, growing the slab's
// allocation if it needs more (hipFree / hipMalloc: synchronous, only when the slab grows).
hipError_t set_far_geometry(Plan& P, double kmax) {
  const FarGeom g = far_geometry(P, kmax, P.M1);
  const size_t nfar = (size_t)g.Mf1 * g.Mf2 * g.S;
  const size_t bytes = (size_t)P.nfo * nfar * P.esize;
  if (bytes > P.far_cap) {
    if (P.ws) return hipErrorInvalidValue;   // callers check the workspace's kmax first
    if (P.far) {
      hipError_t e = hipFree(P.far);
      if (e != hipSuccess) return e;
    }
    P.far = nullptr;
    P.far_cap = 0;
    hipError_t e = hipMalloc(&P.far, bytes);
    if (e != hipSuccess) return e;
    P.far_cap = bytes;
  }
  if (P.gridI_bytes) {
    // the far slab's copy in the gather's layout (node quads of the complex64 G, or the fields
    // interleaved per node)
    const size_t bi = (size_t)(P.nf > 1 ? P.nfo : 4) * nfar * P.esize;
    if (bi > P.farI_cap) {
      if (P.ws) return hipErrorInvalidValue;
      if (P.farI) {
        hipError_t e = hipFree(P.farI);
        if (e != hipSuccess) return e;
      }
      P.farI = nullptr;
      P.farI_cap = 0;
      hipError_t e = hipMalloc(&P.farI, bi);
      if (e != hipSuccess) return e;
      P.farI_cap = bi;
    }
  }
  P.Mf1 = g.Mf1;
  P.Mf2 = g.Mf2;
  P.S = g.S;
  P.fp = g.P;
  P.hf = g.hf;
  P.fz0 = P.p.c - (g.P / 2 - 1) * g.hf;
  P.nfar = nfar;
  return hipSuccess;
}

// Wood anomaly: beta_n = 0 for some mode n (Section 1).  Only lattice points with
// |xi_perp| within 1 of k can come close.
// Entries of the H table on rho = (m - 4) dh that cover |xi| over the grid's modes.
int htab_size(const Plan& P, double a1, double a2) {
  const double e1 = P.M1 / 2 + fabs(a1) + 1.0, e2 = P.M2 / 2 + fabs(a2) + 1.0;
  const double e3 = (P.M3 / 2 + 1.0) * M_PI / P.p.c_tilde;
  return (int)(sqrt(e1 * e1 + e2 * e2 + e3 * e3) / P.hd) + 16;
}

// The far slab for instances up to kmax; a plan on a caller's workspace cannot grow it.
qpgf_status far_for(Plan& P, double kmax) {
  if (P.ws && !(kmax <= P.ws_kmax))
    return fail(QPGF_E_SIZE, "the plan's workspace holds the far slab of wavenumbers up to " +
                                 std::to_string(P.ws_kmax) + "; set a larger workspace");
  HIP_TRY(set_far_geometry(P, kmax));
  return QPGF_OK;
}

// Calls of more targets than a caller's workspace was sized for are refused.
qpgf_status targets_fit(const Plan& P, int64_t T) {
  if (P.ws && T > P.ws_T)
    return fail(QPGF_E_SIZE, "the plan's workspace holds the scratch of " + std::to_string(P.ws_T) +
                                 " targets per call; set a larger workspace");
  return QPGF_OK;
}

qpgf_status check_instance_m1(const Plan& P, double k, double a1, double a2, int M1);
qpgf_status check_instance(const Plan& P, double k, double a1, double a2) {
  return check_instance_m1(P, k, a1, a2, P.M1);
}

qpgf_status check_instance_m1(const Plan& P, double k, double a1, double a2, int M1) {
  (void)M1;
  if (!(k > 0.0) || !std::isfinite(k) || !std::isfinite(a1) || !std::isfinite(a2))
    return fail(QPGF_E_ARG, "need finite k > 0 and finite alpha");
  // the special coefficients beta = -+j pi / c~ are evaluated by the fills (Sections 2.1 / 3.1)
  const double wt = P.p.wood_tol;
  double minb = 1e300;
  if (P.dim == 2) {
    for (long n = (long)floor(-k - a1) - 1; n <= (long)ceil(k - a1) + 1; ++n) {
      double rho = fabs(a1 + n);
      minb = std::min(minb, sqrt(fabs((k - rho) * (k + rho))));
    }
  } else {
    for (long n1 = (long)floor(-k - a1) - 1; n1 <= (long)ceil(k - a1) + 1; ++n1)
      for (long n2 = (long)floor(-k - a2) - 1; n2 <= (long)ceil(k - a2) + 1; ++n2) {
        double rho = sqrt((a1 + n1) * (a1 + n1) + (a2 + n2) * (a2 + n2));
        minb = std::min(minb, sqrt(fabs((k - rho) * (k + rho))));
      }
  }
  if (minb < wt) {
    char buf[160];
    snprintf(buf, sizeof buf, "Wood anomaly: min |beta| = %.3e < wood_tol = %.3e", minb, wt);
    return fail(QPGF_E_WOOD, buf);
  }
  return QPGF_OK;
}

// Whether some coefficient of the grid (x1 index within M1, transverse index within Mt) has
// a propagating beta within special_tol of |J| (J = j pi / c~): only then do the fills compile
// in the special-case path.  A little wider than the fills' own test, so that rounding
// cannot put a coefficient on the other side.
bool has_special(const Plan& P, double k, double a1, double a2, int M1) {
  const long double tol = (long double)P.p.special_tol * 1.01L + 1e-12L;
  const long double step = (long double)M_PI / P.p.c_tilde;
  const long Nt = P.Mt / 2;
  auto near_J = [&](long double rho) -> bool {
    if (rho >= k) return false;
    const long double b = sqrtl(((long double)k - rho) * ((long double)k + rho));
    long j = (long)floorl(b / step);
    for (long jj = j; jj <= j + 1; ++jj)
      if (jj <= Nt && fabsl(b - jj * step) < tol) return true;
    return false;
  };
  const long lo1 = std::max((long)floor(-k - a1) - 1, (long)(-M1 / 2)), hi1 = std::min((long)ceil(k - a1) + 1, (long)(M1 / 2 - 1));
  if (P.dim == 2) {
    for (long n = lo1; n <= hi1; ++n)
      if (near_J(fabsl((long double)a1 + n))) return true;
    return false;
  }
  const long lo2 = std::max((long)floor(-k - a2) - 1, (long)(-P.M2 / 2)), hi2 = std::min((long)ceil(k - a2) + 1, (long)(P.M2 / 2 - 1));
  for (long n1 = lo1; n1 <= hi1; ++n1)
    for (long n2 = lo2; n2 <= hi2; ++n2) {
      const long double e1 = (long double)a1 + n1, e2 = (long double)a2 + n2;
      if (near_J(sqrtl(e1 * e1 + e2 * e2))) return true;
    }
  return false;
}

qpgf_status run_prepare(Plan& P, double k, double a1, double a2, int stage, double k2 = 0.0) {
  if (!P.grid) return fail(QPGF_E_ARG, "the plan has no grid (a failed qpgf_plan_set_workspace): set one again");
  qpgf_status st = check_instance(P, k, a1, a2);
  if (st != QPGF_OK) return st;
  if (P.p.kind == QPGF_KIND_G2D_HESS_DIFF) {
    st = check_instance(P, k2, a1, a2);
    if (st != QPGF_OK) return st;
  }
  st = far_for(P, std::max(k, k2));
  if (st != QPGF_OK) return st;
  P.last_k2 = k2;
  P.spec = has_special(P, k, a1, a2, P.M1) ||
           (P.p.kind == QPGF_KIND_G2D_HESS_DIFF && has_special(P, k2, a1, a2, P.M1));
  P.last_k = k;
  P.last_a1 = a1;
  P.last_a2 = a2;
  P.prepared = false;
  if (P.dim == 3) {
    // H table must cover |xi| over the grid's modes (allocated at creation for |alpha_i| <= 1)
    const int need = htab_size(P, a1, a2);
    if (need > P.hn) {
      if (P.htab) HIP_TRY(hipFree(P.htab));
      P.htab = nullptr;
      HIP_TRY(hipMalloc(reinterpret_cast<void**>(&P.htab), (size_t)need * sizeof(double2)));
      P.hn = need;
    }
    KernelTimer t(P, QPGF_T_HTABLE);
    HIP_TRY(launch_htable(P, k));
  }
  // from stage 1 on, the 3D fill also runs the transverse transform when its pencils fit in LDS
  const bool fused = stage >= 1 && fill_fuses_transverse(P);
  {
    KernelTimer t(P, QPGF_T_FILL);
    HIP_TRY(launch_fill(P, k, a1, a2, fused));
  }
  if (stage >= 1 && !fused) {
    const long nf = P.nf;
    KernelTimer t(P, QPGF_T_FFT_T);
    if (P.dim == 2) {
      // transverse axis j2: stride M1, one batch per j1
      HIP_TRY(launch_fft(P, P.grid, P.M2, P.M1, (long)P.M1 * nf, P.M1, 1, (long)P.ncell));
    } else {
      const long plane = (long)P.M1 * P.M2;
      HIP_TRY(launch_fft(P, P.grid, P.M3, plane, plane * nf, plane, 1, (long)P.ncell));
    }
  }
  if (stage >= 2) {
    const long nf = P.nf;
    if (P.dim == 3) {
      // periodic axis x2 (columns of each slice)
      KernelTimer t(P, QPGF_T_FFT_2);
      HIP_TRY(launch_fft(P, P.grid, P.M2, P.M1, (long)P.M1 * P.M3 * nf, P.M1, 1, (long)P.M1 * P.M2));
    }
    {
      KernelTimer t(P, QPGF_T_FFT_1);
      HIP_TRY(launch_fft(P, P.grid, P.M1, 1, (long)P.M2 * P.M3 * nf, 1, 0, P.M1));
    }
    {
      KernelTimer t(P, QPGF_T_FAR);
      HIP_TRY(launch_far(P, k, a1, a2));
    }
    {
      // the far slab on its own periodic grid Mf1 x Mf2: rows (x1; in 3D the far fill above has
      // already run the x2 columns), or the x2 columns where the Maxwell far fill ran the rows
      KernelTimer t(P, QPGF_T_FAR_FFT);
      if (far_rows_in_fill(P))
        HIP_TRY(launch_fft_far_cols(P, k, a2));
      else if (P.dim == 3 && P.nfo == 1)
        HIP_TRY(launch_fft_far_rows(P, k, a1));
      else
        HIP_TRY(launch_fft(P, P.far, P.Mf1, 1, (long)P.Mf2 * P.S * P.nfo, 1, 0, P.Mf1));
    }
    if (P.dim == 2 && P.gridI) {
      // the gather reads a stencil row (of all fields) as one contiguous, aligned run
      KernelTimer t(P, QPGF_T_LAYOUT);
      HIP_TRY(launch_interleave2d(P));
    }
    P.prepared = true;
  }
  return QPGF_OK;
}

qpgf_status check_plan(const qpgf_plan* plan, int kind) {
  if (!plan) return fail(QPGF_E_ARG, "plan is NULL");
  if (kind >= 0 && plan->P.p.kind != kind) return fail(QPGF_E_ARG, "entry point does not match the plan kind");
  return QPGF_OK;
}

qpgf_status run_evaluate(Plan& P, const double* x, int64_t T, void* out, uint8_t* flags) {
  if (T < 0) return fail(QPGF_E_ARG, "T < 0");
  if (T == 0) return QPGF_OK;
  if (!x || !out) return fail(QPGF_E_ARG, "x and out must be non-NULL device pointers");
  if (!P.prepared) return fail(QPGF_E_ARG, "evaluate before a complete prepare");
  if (T > (int64_t)0x7fffffff) return fail(QPGF_E_SIZE, "at most 2^31 - 1 targets per call");
  qpgf_status st = targets_fit(P, T);
  if (st != QPGF_OK) return st;
  HIP_TRY(launch_gather(P, x, T, out, flags));
  return QPGF_OK;
}

// The workspace's parts, each 256-byte aligned: near grid, its interleaved copy, the far slab
// of the largest instance (kmax), the target scratch of T targets.
struct WsLayout {
  size_t grid = 0, gridI = 0, far = 0, farI = 0, targets = 0, total = 0;
  int nkeys = 0;
};
size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }
WsLayout ws_layout(const Plan& P, double kmax, int64_t T) {
  WsLayout L;
  L.grid = al256((size_t)P.nf * P.ncell * P.esize);
  L.gridI = al256(P.gridI_bytes);
  const FarGeom g = far_geometry(P, kmax, P.M1);
  const size_t nfar = (size_t)g.Mf1 * g.Mf2 * g.S;
  L.far = al256((size_t)P.nfo * nfar * P.esize);
  L.farI = P.gridI_bytes ? al256((size_t)(P.nf > 1 ? P.nfo : 4) * nfar * P.esize) : 0;
  L.nkeys = bin_keys_bound(P, g.Mf1, g.Mf2, g.S, g.P);
  TargetScratch t;
  L.targets = carve_target_scratch(P, nullptr, T, L.nkeys, t);
  L.total = L.grid + L.gridI + L.far + L.farI + L.targets;
  return L;
}

qpgf_status check_ws_args(double kmax, int64_t T) {
  if (!(kmax >= 0.0) || !std::isfinite(kmax)) return fail(QPGF_E_ARG, "kmax must be finite and >= 0");
  if (T < 0 || T > (int64_t)0x7fffffff) return fail(QPGF_E_ARG, "max_targets must be in [0, 2^31 - 1]");
  return QPGF_OK;
}

void drain_timers(Plan& P) {
  for (auto& e : P.pending) {
    float ms = 0.f;
    if (hipEventSynchronize(e.b) == hipSuccess && hipEventElapsedTime(&ms, e.a, e.b) == hipSuccess) {
      P.t_ms[e.id] += ms;
      P.t_n[e.id] += 1;
    }
    (void)hipEventDestroy(e.a);
    (void)hipEventDestroy(e.b);
  }
  P.pending.clear();
}

// Fixed target scratch of qpgf_evaluate_noalloc: each GPU the library runs on holds its own copy
// until the process ends.  Host code never uses the name for memory: the per-device address
// comes from hipGetSymbolAddress (scratch_address).
constexpr size_t kNoAllocScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

}  // namespace

static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {

// The device address of the current GPU's copy of the scratch, looked up on the first call on
// each device (with that device current) and kept.
qpgf_status scratch_address(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(QPGF_E_UNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(QPGF_E_HIP, "hipGetSymbolAddress returned NULL for the fixed scratch");
    g_scratch_ptr[dev] = static_cast<char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return QPGF_OK;
}

}  // namespace

extern "C" {

void qpgf_params_default(qpgf_params* p, int kind, int prec, int m1, int m2, int m3) {
  if (!p) return;
  std::memset(p, 0, sizeof *p);
  p->kind = kind;
  p->prec = prec;
  p->m1 = m1;
  p->m2 = m2;
  p->m3 = m3;
  p->c = 0.6;
  p->c_tilde = 1.0;
  p->eps = 0.2;
  p->quad_q = 64;
  p->far_h = 0.0;   // automatic: see far_geometry
  p->far_zmax = p->c_tilde;
  p->wood_tol = 1e-3;
  p->special_tol = 1e-2;
  p->lattice_rmin = 0.0;
  p->sing_order = 1;
  p->ring_interp = 0;
}

qpgf_status qpgf_plan_create(const qpgf_params* p, qpgf_plan** out) {
  g_err.clear();
  if (!out) return fail(QPGF_E_ARG, "out is NULL");
  *out = nullptr;
  qpgf_status st = validate(p);
  if (st != QPGF_OK) return st;
  auto* plan = new (std::nothrow) qpgf_plan();
  if (!plan) return fail(QPGF_E_NOMEM, "host allocation failed");
  Plan& P = plan->P;
  P.p = *p;
  P.dim = kind_is_2d(p->kind) ? 2 : 3;
  P.nf = (p->kind == QPGF_KIND_MAXWELL3D)       ? (p->maxwell_trace ? kMxT : kMxF)
         : (p->kind == QPGF_KIND_G2D_HESS_DIFF) ? 3
         : (p->kind == QPGF_KIND_G2D_GRAD)      ? 2
                                                : 1;
  P.M1 = p->m1;
  P.M2 = p->m2;
  P.M3 = (P.dim == 3) ? p->m3 : 1;
  P.Mt = (P.dim == 3) ? P.M3 : P.M2;
  P.esize = (p->prec == QPGF_C128) ? 16 : 8;
  P.nfo = p->kind == QPGF_KIND_MAXWELL3D ? kMxO : P.nf;
  P.ncell = (size_t)P.M1 * P.M2 * P.M3;

  auto bail = [&](qpgf_status s) {
    free_plan(P);
    delete plan;
    return s;
  };
#define PLAN_TRY(call)                                     \
  do {                                                     \
    hipError_t e_ = (call);                                \
    if (e_ != hipSuccess) return bail(hip_fail(e_, #call)); \
  } while (0)
#define PLAN_ST(expr)                  \
  do {                                 \
    qpgf_status s_ = (expr);           \
    if (s_ != QPGF_OK) return bail(s_); \
  } while (0)

  PLAN_TRY(hipGetDevice(&P.device));
  PLAN_TRY(hipMalloc(&P.grid, P.nf * P.ncell * P.esize));
  PLAN_TRY(set_far_geometry(P, 0.0));   // the smallest slab; instances that need more grow it
  if (P.dim == 3) {
    P.hn = htab_size(P, 1.0, 1.0);
    PLAN_TRY(hipMalloc(reinterpret_cast<void**>(&P.htab), (size_t)P.hn * sizeof(double2)));
  }
  // complex64 G: each node's quad of x1-neighbours (4 values, 32 bytes) while the quads stay about
  // L2-sized (measured: 4.4 MB of quads read 30 % faster than the grid row by row, 8.8 MB slower)
  const bool quads = P.dim == 2 && P.nf == 1 && P.p.prec == QPGF_C64 && 32 * P.ncell <= (5u << 20);
  if (P.dim == 2 && (P.nf > 1 || quads)) {
    // derivative kinds: the near fields interleaved per node; the complex64 G: node quads
    const size_t per = P.nf > 1 ? (size_t)P.nf : 4;
    P.gridI_bytes = per * P.ncell * P.esize;
    PLAN_TRY(hipMalloc(&P.gridI, P.gridI_bytes));
  }

  const int Q = p->quad_q;
  std::vector<long double> gx, gw;
  gauss_legendre(Q, gx, gw);
  // X'-integral rule on [c, (c + c~)/2]: X'(x) = -S'((x - c)/w)/w, w = (c~ - c)/2
  {
    const long double c = p->c, w = 0.5L * (p->c_tilde - p->c);
    std::vector<double> xq(Q), wxq(Q), wXq(Q);
    for (int q = 0; q < Q; ++q) {
      long double x = c + 0.5L * w * (gx[q] + 1.0L);
      long double u = (x - c) / w;
      xq[q] = (double)x;
      wxq[q] = (double)(0.5L * w * gw[q] * (-(long double)smooth_S1((double)u) / w));
      wXq[q] = (double)(0.5L * w * gw[q] * (1.0L - (long double)smooth_S((double)u)));
    }
    PLAN_ST(upload(&P.xq, xq));
    PLAN_ST(upload(&P.wxq, wxq));
    PLAN_ST(upload(&P.wXq, wXq));
    const int Nt = P.Mt / 2;
    std::vector<double2> cs((size_t)(Nt + 1) * Q);
    for (int j = 0; j <= Nt; ++j)
      for (int q = 0; q < Q; ++q) {
        long double a = (long double)j * kPiL / p->c_tilde * (long double)xq[q];
        cs[(size_t)j * Q + q] = make_double2((double)cosl(a), (double)sinl(a));
      }
    PLAN_ST(upload(&P.cs, cs));
  }
  // radial rule on [eps, 2 eps] with Y', Y'' at the nodes.  Its integrands carry J0(|eta| r),
  // sin(rho r) up to the grid's largest frequency (2D: |eta| of the corner mode; 3D: the end of the
  // H table); measured, the rule reaches rounding with about 0.065 |eta| + 16 nodes (80 at |eta| =
  // 1043, the corner of 2048 x 128), so it takes max(quad_q, 0.07 |eta| + 24) of them.
  const double eta_max = P.dim == 2 ? std::hypot(P.M1 / 2 + 1.0, (P.M2 / 2) * M_PI / p->c_tilde) : P.hn * P.hd;
  P.Qr = std::max(Q, 8 * (int)std::ceil((0.07 * eta_max + 24.0) / 8.0));
  const int Qr = P.Qr;
  std::vector<long double> rx, rw;
  gauss_legendre(Qr, rx, rw);
  std::vector<double> rq(Qr), wrq(Qr), y1q(Qr), y2q(Qr);
  {
    const long double e = p->eps;
    for (int q = 0; q < Qr; ++q) {
      long double r = e + 0.5L * e * (rx[q] + 1.0L);
      rq[q] = (double)r;
      wrq[q] = (double)(0.5L * e * rw[q]);
      y1q[q] = cut_Y1(rq[q], p->eps);
      y2q[q] = cut_Y2(rq[q], p->eps);
    }
    PLAN_ST(upload(&P.rq, rq));
    PLAN_ST(upload(&P.wrq, wrq));
    PLAN_ST(upload(&P.y1q, y1q));
    PLAN_ST(upload(&P.y2q, y2q));
  }
  // twiddles e^{+2 pi i j / NT}
  {
    // every transform length (far slabs grow with k) divides NT and reads this table with a stride;
    // one octant is evaluated, the rest follows by symmetry: quadrant turns multiply by i, and
    // within a quadrant e^{i(pi/2 - t)} swaps cos and sin
    const int NT = kTwiddles, NQ = NT / 4;
    P.ntw = NT;
    std::vector<long double> cb(NQ / 2 + 1), sb(NQ / 2 + 1);
    for (int q = 0; q <= NQ / 2; ++q) {
      const long double a = 2.0L * kPiL * q / NT;
      cb[q] = cosl(a);
      sb[q] = sinl(a);
    }
    std::vector<double2> tw(NT);
    std::vector<float2> twf(NT);
    for (int j = 0; j < NT; ++j) {
      const int quad = j / NQ, q = j - quad * NQ;
      long double c = q <= NQ / 2 ? cb[q] : sb[NQ - q], sn = q <= NQ / 2 ? sb[q] : cb[NQ - q];
      for (int t = 0; t < quad; ++t) {
        const long double c0 = c;
        c = -sn;
        sn = c0;
      }
      tw[j] = make_double2((double)c, (double)sn);
      twf[j] = make_float2((float)c, (float)sn);
    }
    PLAN_ST(upload(&P.tw, tw));
    PLAN_ST(upload(&P.twf, twf));
  }
  const bool ho = p->kind == QPGF_KIND_G2D && p->sing_order > 1;
  if (p->kind == QPGF_KIND_G2D_GRAD || p->kind == QPGF_KIND_G2D_HESS_DIFF || ho) {
    // derivative and higher-order tables: Gauss-Legendre rule on [eps, 2 eps] for |eta| up to the grid's corner
    // (about |eta| eps nodes beyond the plain rule resolve the Bessel oscillations)
    const double e1 = P.M1 / 2, e2 = (P.M2 / 2) * M_PI / p->c_tilde;
    const int Qg = std::max(Q, (int)std::ceil(std::sqrt(e1 * e1 + e2 * e2) * p->eps) + 64);
    std::vector<long double> hx, hw;
    gauss_legendre(Qg, hx, hw);
    std::vector<double> rg(Qg), wyg(Qg);
    const long double e = p->eps;
    for (int q = 0; q < Qg; ++q) {
      rg[q] = (double)(e + 0.5L * e * (hx[q] + 1.0L));
      wyg[q] = (double)(0.5L * e * hw[q] * (long double)cut_Y(rg[q], p->eps));
    }
    double *drg = nullptr, *dwyg = nullptr;
    PLAN_ST(upload(&drg, rg));
    qpgf_status su = upload(&dwyg, wyg);
    if (su != QPGF_OK) {
      (void)hipFree(drg);
      return bail(su);
    }
    hipError_t e2r;
    if (ho) {
      e2r = hipMalloc(reinterpret_cast<void**>(&P.E2), 4 * P.ncell * sizeof(double));
      if (e2r == hipSuccess) e2r = launch_sing2d_ho(P, Qg, drg, dwyg);
    } else {
      const bool grad = p->kind == QPGF_KIND_G2D_GRAD;
      e2r = hipMalloc(reinterpret_cast<void**>(&P.D2), (grad ? 8 : 6) * P.ncell * sizeof(double));
      if (e2r == hipSuccess) e2r = grad ? launch_sing2d_grad(P, Qg, drg, dwyg) : launch_sing2d_hess(P, Qg, drg, dwyg);
    }
    if (e2r == hipSuccess) e2r = hipDeviceSynchronize();
    (void)hipFree(drg);
    (void)hipFree(dwyg);
    PLAN_TRY(e2r);
  }
  if (p->kind == QPGF_KIND_G2D) {
    // Phi_1(r) = (2 + ln r) Y'(r)/r + Y''(r) ln r at the radial nodes, times the weights
    std::vector<double> wphi(Qr);
    long double f1tail = 0.0L;
    for (int q = 0; q < Qr; ++q) {
      long double r = rq[q], lr = logl(r);
      wphi[q] = (double)(wrq[q] * ((2.0L + lr) * y1q[q] / r + y2q[q] * lr));
      f1tail += (long double)wrq[q] * r * lr * cut_Y(rq[q], p->eps);
    }
    // F1_0 = -A2 int_0^{2eps} t ln t Y(t) dt, with int_0^eps t ln t dt = eps^2 (ln eps / 2 - 1/4)
    const long double e = p->eps;
    const long double A2 = 1.0L / (2.0L * sqrtl(kPiL * p->c_tilde));
    const double f1zero = (double)(-A2 * (e * e * (logl(e) / 2.0L - 0.25L) + f1tail));
    double* dphi = nullptr;
    PLAN_ST(upload(&dphi, wphi));
    PLAN_TRY(hipMalloc(reinterpret_cast<void**>(&P.F1), P.ncell * sizeof(double2)));
    PLAN_TRY(hipMalloc(reinterpret_cast<void**>(&P.F2), P.ncell * sizeof(double2)));
    double* save = P.wrq;   // k_sing2d takes the combined weights in place of wrq
    P.wrq = dphi;
    hipError_t e2 = launch_sing2d(P, f1zero);
    P.wrq = save;
    if (e2 == hipSuccess) e2 = hipDeviceSynchronize();
    (void)hipFree(dphi);
    PLAN_TRY(e2);
  }
  PLAN_TRY(hipDeviceSynchronize());
#undef PLAN_TRY
#undef PLAN_ST
  *out = plan;
  return QPGF_OK;
}

void qpgf_plan_destroy(qpgf_plan* plan) {
  if (!plan) return;
  if (plan->P.stream) (void)hipStreamSynchronize(plan->P.stream);
  else (void)hipDeviceSynchronize();
  drain_timers(plan->P);
  free_plan(plan->P);
  delete plan;
}

qpgf_status qpgf_plan_set_stream(qpgf_plan* plan, void* hip_stream) {
  if (!plan) return fail(QPGF_E_ARG, "plan is NULL");
  plan->P.stream = static_cast<hipStream_t>(hip_stream);
  return QPGF_OK;
}

qpgf_status qpgf_plan_get_info(const qpgf_plan* plan, qpgf_plan_info* info) {
  if (!plan || !info) return fail(QPGF_E_ARG, "plan and info must be non-NULL");
  const Plan& P = plan->P;
  info->kind = P.p.kind;
  info->prec = P.p.prec;
  info->m1 = P.M1;
  info->m2 = P.M2;
  info->m3 = P.dim == 3 ? P.M3 : 0;
  info->far_slices = P.S;
  info->far_h = P.hf;
  info->c = P.p.c;
  info->c_tilde = P.p.c_tilde;
  info->eps = P.p.eps;
  info->n_fields = P.nf;
  info->grid_bytes = P.ncell * P.esize;
  info->far_grid_bytes = P.nfar * P.esize;
  info->far_m1 = P.Mf1;
  info->far_m2 = P.Mf2;
  info->far_fields = P.nfo;
  info->far_points = P.fp;
  info->far_points_t = (P.dim == 3 && P.p.prec == QPGF_C128 && P.nf == 1 && far7_ok(P)) ? 7 : P.fp;
  return QPGF_OK;
}

qpgf_status qpgf_prepare(qpgf_plan* plan, double k, double a1, double a2) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  if (plan->P.p.kind == QPGF_KIND_G2D_HESS_DIFF)
    return fail(QPGF_E_ARG, "a plan of kind G2D_HESS_DIFF takes two wavenumbers: qpgf_prepare_hess_diff");
  return run_prepare(plan->P, k, a1, plan->P.dim == 3 ? a2 : 0.0, 2);
}

qpgf_status qpgf_prepare_stage(qpgf_plan* plan, double k, double a1, double a2, int stage) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  if (plan->P.p.kind == QPGF_KIND_G2D_HESS_DIFF)
    return fail(QPGF_E_ARG, "a plan of kind G2D_HESS_DIFF takes two wavenumbers: qpgf_prepare_hess_diff");
  if (stage < 0 || stage > 2) return fail(QPGF_E_ARG, "stage must be 0, 1 or 2");
  return run_prepare(plan->P, k, a1, plan->P.dim == 3 ? a2 : 0.0, stage);
}

qpgf_status qpgf_prepare_hess_diff(qpgf_plan* plan, double k1, double k2, double alpha, int stage) {
  g_err.clear();
  qpgf_status st = check_plan(plan, QPGF_KIND_G2D_HESS_DIFF);
  if (st != QPGF_OK) return st;
  if (stage < 0 || stage > 2) return fail(QPGF_E_ARG, "stage must be 0, 1 or 2");
  return run_prepare(plan->P, k1, alpha, 0.0, stage, k2);
}

qpgf_status qpgf_evaluate(qpgf_plan* plan, const double* x, int64_t T, void* out, uint8_t* flags) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  return run_evaluate(plan->P, x, T, out, flags);
}

static qpgf_status both(qpgf_plan* plan, int kind, double k, double a1, double a2, const double* x, int64_t T,
                        void* out, uint8_t* flags, double k2 = 0.0) {
  g_err.clear();
  qpgf_status st = check_plan(plan, kind);
  if (st != QPGF_OK) return st;
  Plan& P = plan->P;
  if (T < 0) return fail(QPGF_E_ARG, "T < 0");
  if (T > 0 && (!x || !out)) return fail(QPGF_E_ARG, "x and out must be non-NULL device pointers");
  if (T > (int64_t)0x7fffffff) return fail(QPGF_E_SIZE, "at most 2^31 - 1 targets per call");
  st = targets_fit(P, T);
  if (st != QPGF_OK) return st;
  // The binning of the targets depends on the targets and the grid geometry
  // only: it runs on a second stream while the grids are prepared (fork after
  // the work already on the plan's stream, join before the gather).
  const bool overlap = T > 0 && gather_uses_bins(P, T);
  if (overlap) {
    // the tile keys of far targets depend on the instance's far slab
    if (!std::isfinite(k) || !std::isfinite(k2)) return fail(QPGF_E_ARG, "need finite k");
    st = far_for(P, std::max(k, k2));
    if (st != QPGF_OK) return st;
    if (!P.side) HIP_TRY(hipStreamCreateWithFlags(&P.side, hipStreamNonBlocking));
    if (!P.ev_fork) HIP_TRY(hipEventCreateWithFlags(&P.ev_fork, hipEventDisableTiming));
    if (!P.ev_join) HIP_TRY(hipEventCreateWithFlags(&P.ev_join, hipEventDisableTiming));
    HIP_TRY(hipEventRecord(P.ev_fork, P.stream));
    HIP_TRY(hipStreamWaitEvent(P.side, P.ev_fork, 0));
    HIP_TRY(launch_bin3d(P, x, T, P.side));
    HIP_TRY(hipEventRecord(P.ev_join, P.side));
  }
  st = run_prepare(P, k, a1, a2, 2, k2);
  if (overlap) {
    // the plan's stream owns the bin scratch again, also when the preparation failed
    HIP_TRY(hipStreamWaitEvent(P.stream, P.ev_join, 0));
  }
  if (st != QPGF_OK) return st;
  if (overlap) {
    HIP_TRY(launch_gather_binned(P, x, T, out, flags));
    return QPGF_OK;
  }
  return run_evaluate(P, x, T, out, flags);
}

qpgf_status qpgf_g2d(qpgf_plan* plan, double k, double alpha, const double* x, int64_t T, void* out,
                     uint8_t* flags) {
  return both(plan, QPGF_KIND_G2D, k, alpha, 0.0, x, T, out, flags);
}

qpgf_status qpgf_g2d_grad(qpgf_plan* plan, double k, double alpha, const double* x, int64_t T, void* out,
                          uint8_t* flags) {
  return both(plan, QPGF_KIND_G2D_GRAD, k, alpha, 0.0, x, T, out, flags);
}

qpgf_status qpgf_g2d_hess_diff(qpgf_plan* plan, double k1, double k2, double alpha, const double* x, int64_t T,
                               void* out, uint8_t* flags) {
  return both(plan, QPGF_KIND_G2D_HESS_DIFF, k1, alpha, 0.0, x, T, out, flags, k2);
}

qpgf_status qpgf_gd3d(qpgf_plan* plan, double k, double a1, double a2, const double* x, int64_t T, void* out,
                      uint8_t* flags) {
  return both(plan, QPGF_KIND_GD3D, k, a1, a2, x, T, out, flags);
}

qpgf_status qpgf_maxwell3d(qpgf_plan* plan, double k, double a1, double a2, const double* x, int64_t T,
                           void* out, uint8_t* flags) {
  return both(plan, QPGF_KIND_MAXWELL3D, k, a1, a2, x, T, out, flags);
}

qpgf_status qpgf_evaluate_noalloc(qpgf_plan* plan, const double* x, int64_t T, void* out, uint8_t* flags) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  Plan& P = plan->P;
  if (T < 0) return fail(QPGF_E_ARG, "T < 0");
  if (T == 0) return QPGF_OK;
  if (!x || !out) return fail(QPGF_E_ARG, "x and out must be non-NULL device pointers");
  if (!P.prepared) return fail(QPGF_E_ARG, "evaluate before a complete prepare");
  if (T > (int64_t)0x7fffffff) return fail(QPGF_E_SIZE, "at most 2^31 - 1 targets per call");
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != P.device) return fail(QPGF_E_ARG, "make the plan's device current");
  const int nkeys = bin_keys_bound(P, P.Mf1, P.Mf2, P.S, P.fp);
  TargetScratch mine;
  if (carve_target_scratch(P, nullptr, T, nkeys, mine) > kNoAllocScratchBytes) {
    int64_t lo = 0, hi = T;   // the most targets whose scratch fits
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (carve_target_scratch(P, nullptr, mid, nkeys, mine) <= kNoAllocScratchBytes) lo = mid;
      else hi = mid - 1;
    }
    return fail(QPGF_E_SIZE, "qpgf_evaluate_noalloc: at most " + std::to_string(lo) +
                                 " targets per call fit the fixed scratch of this plan's geometry (64 MiB)");
  }
  char* base = nullptr;
  st = scratch_address(dev, &base);
  if (st != QPGF_OK) return st;
  carve_target_scratch(P, base, T, nkeys, mine);
  // the plan's own scratch is set aside for the call; timers (which create events) are off
  const bool timing = P.timing;
  P.timing = false;
  std::swap(P.ts, mine);
  const hipError_t e = launch_gather(P, x, T, out, flags);
  std::swap(P.ts, mine);
  P.timing = timing;
  P.bt_T = -1;
  P.bt_x = nullptr;
  if (e != hipSuccess) return hip_fail(e, "launch_gather (fixed scratch)");
  return QPGF_OK;
}

qpgf_status qpgf_plan_workspace_bytes(const qpgf_plan* plan, double kmax, int64_t max_targets, size_t* bytes) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  if (!bytes) return fail(QPGF_E_ARG, "bytes is NULL");
  st = check_ws_args(kmax, max_targets);
  if (st != QPGF_OK) return st;
  *bytes = ws_layout(plan->P, kmax, max_targets).total;
  return QPGF_OK;
}

qpgf_status qpgf_plan_set_workspace(qpgf_plan* plan, void* ptr, size_t bytes, double kmax, int64_t max_targets) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  Plan& P = plan->P;
  if (ptr) {
    st = check_ws_args(kmax, max_targets);
    if (st != QPGF_OK) return st;
    if (reinterpret_cast<uintptr_t>(ptr) % 256) return fail(QPGF_E_ARG, "the workspace must be 256-byte aligned");
  } else if (bytes) {
    return fail(QPGF_E_ARG, "a NULL workspace must have 0 bytes");
  }
  const WsLayout L = ptr ? ws_layout(P, kmax, max_targets) : WsLayout{};
  if (ptr && bytes < L.total)
    return fail(QPGF_E_SIZE, "the workspace needs " + std::to_string(L.total) + " bytes (qpgf_plan_workspace_bytes)");
  // nothing in flight may still use the arrays being replaced
  HIP_TRY(hipStreamSynchronize(P.stream));
  if (P.side) HIP_TRY(hipStreamSynchronize(P.side));
  drain_timers(P);
  if (!P.ws) {
    for (void* q : {P.grid, P.gridI, P.far, P.farI})
      if (q) HIP_TRY(hipFree(q));
  }
  free_target_scratch(P.ts);
  P.grid = P.gridI = P.far = P.farI = nullptr;
  P.far_cap = 0;
  P.farI_cap = 0;
  P.ws = nullptr;
  P.ws_bytes = 0;
  P.ws_kmax = 0.0;
  P.ws_T = 0;
  P.prepared = false;
  P.bt_T = -1;
  P.bt_x = nullptr;
  if (ptr) {
    char* b = static_cast<char*>(ptr);
    P.ws = b;
    P.ws_bytes = bytes;
    P.ws_kmax = kmax;
    P.ws_T = max_targets;
    P.grid = b;
    P.gridI = P.gridI_bytes ? b + L.grid : nullptr;
    P.far = b + L.grid + L.gridI;
    P.far_cap = L.far;
    P.farI = L.farI ? b + L.grid + L.gridI + L.far : nullptr;
    P.farI_cap = L.farI;
    carve_target_scratch(P, b + L.grid + L.gridI + L.far + L.farI, max_targets, L.nkeys, P.ts);
  } else {
    // the plan's own arrays again (the target scratch grows on demand)
    HIP_TRY(hipMalloc(&P.grid, (size_t)P.nf * P.ncell * P.esize));
    if (P.gridI_bytes) HIP_TRY(hipMalloc(&P.gridI, P.gridI_bytes));
  }
  HIP_TRY(set_far_geometry(P, 0.0));
  return QPGF_OK;
}

}  // extern "C"

// ----------------------------------------------------------------------------
// batched 2D
// ----------------------------------------------------------------------------
namespace {

template <typename V>
hipError_t grow(V** p, size_t& cap, size_t bytes) {
  if (bytes <= cap) return hipSuccess;
  if (*p) (void)hipFree(*p);
  *p = nullptr;
  cap = 0;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(p), bytes);
  if (e == hipSuccess) cap = bytes;
  return e;
}

struct BatchLayout {
  size_t fill_off, far_off, gat_off, segT_off, segR_off, segF_off, bytes;
  long fill_blocks, far_blocks, gat_blocks, segT_blocks, segR_blocks, segF_blocks;
  long lds_T, lds_R, lds_F;   // largest tile * (n + 1) over the segments of each launch
};

size_t align_up(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

extern "C" qpgf_status qpgf_g2d_batched(qpgf_plan* plan, int n_inst, const double* k, const double* alpha,
                                        const int* m1, const int64_t* t_off, const double* x, void* out,
                                        uint8_t* flags) {
  g_err.clear();
  qpgf_status st = check_plan(plan, QPGF_KIND_G2D);
  if (st != QPGF_OK) return st;
  Plan& P = plan->P;
  if (P.p.ring_interp) return fail(QPGF_E_ARG, "ring_interp is not available in qpgf_g2d_batched");
  if (n_inst <= 0 || !k || !alpha || !m1 || !t_off) return fail(QPGF_E_ARG, "need n_inst > 0 and host k, alpha, m1, t_off");
  if (t_off[0] != 0) return fail(QPGF_E_ARG, "t_off[0] must be 0");
  for (int i = 0; i < n_inst; ++i) {
    if (!m1_2d_in(m1[i], 16, P.M1))
      return fail(QPGF_E_SIZE, "m1[i] must be in [16, params.m1]: 2^a r with a >= 1 and r = 1, 3, 5 or 7");
    if (t_off[i + 1] < t_off[i]) return fail(QPGF_E_ARG, "t_off must be non-decreasing");
  }
  const int64_t T = t_off[n_inst];
  if (T > 0 && (!x || !out)) return fail(QPGF_E_ARG, "x and out must be non-NULL device pointers");
  if (T > (int64_t)0x7fffffff) return fail(QPGF_E_SIZE, "at most 2^31 - 1 targets per call");
  for (int i = 0; i < n_inst; ++i) {
    st = check_instance_m1(P, k[i], alpha[i], 0.0, m1[i]);
    if (st != QPGF_OK) {
      g_err = "instance " + std::to_string(i) + ": " + g_err;
      return st;
    }
  }
  // layout of the instance grids and of the descriptors
  const size_t fsz = fill_inst_size(), gsz = gather_inst_size();
  BatchLayout Lo{};
  Lo.fill_off = 0;
  Lo.far_off = align_up(Lo.fill_off + n_inst * fsz);
  Lo.gat_off = align_up(Lo.far_off + n_inst * fsz);
  Lo.segT_off = align_up(Lo.gat_off + n_inst * gsz);
  Lo.segR_off = align_up(Lo.segT_off + n_inst * sizeof(FftSeg));
  Lo.segF_off = align_up(Lo.segR_off + n_inst * sizeof(FftSeg));
  Lo.bytes = align_up(Lo.segF_off + n_inst * sizeof(FftSeg));
  // each instance's far slab on its own geometry (modes and slices follow its wavenumber)
  std::vector<FarGeom> fg(n_inst);
  size_t grid_elems = 0, far_elems = 0;
  for (int i = 0; i < n_inst; ++i) {
    fg[i] = far_geometry(P, k[i], m1[i]);
    grid_elems += (size_t)m1[i] * P.M2;
    far_elems += (size_t)fg[i].Mf1 * fg[i].S;
  }
  HIP_TRY(grow(&P.b_grid, P.b_grid_cap, grid_elems * P.esize));
  HIP_TRY(grow(&P.b_far, P.b_far_cap, far_elems * P.esize));
  if (Lo.bytes > P.b_desc_cap) {
    if (P.b_upload_done) HIP_TRY(hipEventSynchronize(P.b_upload_done));
    if (P.b_host) (void)hipHostFree(P.b_host);
    P.b_host = nullptr;
    if (P.b_desc) (void)hipFree(P.b_desc);
    P.b_desc = nullptr;
    P.b_desc_cap = 0;
    HIP_TRY(hipHostMalloc(&P.b_host, Lo.bytes));
    HIP_TRY(hipMalloc(&P.b_desc, Lo.bytes));
    P.b_desc_cap = Lo.bytes;
    free_batch(P);     // the graph refers to the old descriptor buffer
  }
  if (!P.b_upload_done) HIP_TRY(hipEventCreateWithFlags(&P.b_upload_done, hipEventDisableTiming));
  HIP_TRY(hipEventSynchronize(P.b_upload_done));   // previous upload finished with the staging buffer
  char* h = static_cast<char*>(P.b_host);
  long fb = 0, rb = 0, gb = 0, tb = 0, rrb = 0, frb = 0;
  size_t goff = 0, foff = 0;
  Lo.lds_T = Lo.lds_R = Lo.lds_F = 0;
  for (int i = 0; i < n_inst; ++i) {
    const int M = m1[i], MF = fg[i].Mf1, SF = fg[i].S;
    fill_inst_2d(P, k[i], alpha[i], M, fg[i], (long)goff, (long)foff, fb, h + Lo.fill_off + i * fsz);
    fb += (M + 15) / 16;
    fill_inst_2d(P, k[i], alpha[i], M, fg[i], (long)goff, (long)foff, rb, h + Lo.far_off + i * fsz);
    rb += ((long)MF * SF + 255) / 256;
    gather_inst_2d(P, k[i], alpha[i], M, fg[i], (long)goff, (long)foff, (long)t_off[i], (long)t_off[i + 1], gb,
                   h + Lo.gat_off + i * gsz);
    gb += (long)((t_off[i + 1] - t_off[i] + 255) / 256);
    FftSeg sT{(long)goff, P.M2, (long)M, (long)M, (long)M, 1, 0,
              fft_tile(P, P.M2, false, M), tb};
    tb += (sT.nbatch + sT.tile - 1) / sT.tile;
    // column transforms: padded rows; plus the twiddles when they fit
    Lo.lds_T = std::max(Lo.lds_T, (long)sT.tile * (sT.n + 1) +
                                      (fft_twiddles_in_lds(sT.tile, sT.n + 1, sT.n, P.esize) ? sT.n : 0));
    FftSeg sR{(long)goff, M, 1, (long)P.M2, 1, 0, (long)M, fft_tile(P, M, true, P.M2), rrb};
    rrb += (sR.nbatch + sR.tile - 1) / sR.tile;
    Lo.lds_R = std::max(Lo.lds_R, (long)sR.tile * sR.n + (fft_twiddles_in_lds(sR.tile, sR.n, sR.n, P.esize) ? sR.n : 0));
    FftSeg sF{(long)foff, MF, 1, (long)SF, 1, 0, (long)MF, fft_tile(P, MF, true, SF), frb};
    frb += (sF.nbatch + sF.tile - 1) / sF.tile;
    Lo.lds_F = std::max(Lo.lds_F, (long)sF.tile * sF.n + (fft_twiddles_in_lds(sF.tile, sF.n, sF.n, P.esize) ? sF.n : 0));
    std::memcpy(h + Lo.segT_off + i * sizeof(FftSeg), &sT, sizeof sT);
    std::memcpy(h + Lo.segR_off + i * sizeof(FftSeg), &sR, sizeof sR);
    std::memcpy(h + Lo.segF_off + i * sizeof(FftSeg), &sF, sizeof sF);
    goff += (size_t)M * P.M2;
    foff += (size_t)MF * SF;
  }
  Lo.fill_blocks = fb;
  Lo.far_blocks = rb;
  Lo.gat_blocks = gb;
  Lo.segT_blocks = tb;
  Lo.segR_blocks = rrb;
  Lo.segF_blocks = frb;
  // LDS of one k_fft_multi launch: one in-place buffer for its largest tile * pitch
  if ((size_t)std::max(Lo.lds_T, std::max(Lo.lds_R, Lo.lds_F)) * P.esize > 65536)
    return fail(QPGF_E_SIZE, "FFT tile choice exceeds the LDS of one block");
  const hipStream_t user = P.stream;
  HIP_TRY(hipMemcpyAsync(P.b_desc, P.b_host, Lo.bytes, hipMemcpyHostToDevice, user));
  HIP_TRY(hipEventRecord(P.b_upload_done, user));

  bool spec = false;
  for (int i = 0; i < n_inst && !spec; ++i) spec = has_special(P, k[i], alpha[i], 0.0, m1[i]);
  std::vector<int64_t> sig;
  sig.push_back(n_inst);
  sig.push_back(P.p.prec);
  sig.push_back(spec);
  for (int i = 0; i < n_inst; ++i) {
    sig.push_back(m1[i]);
    sig.push_back(((int64_t)fg[i].Mf1 << 32) | fg[i].S);   // the far slabs' shapes follow k
  }
  for (int i = 0; i <= n_inst; ++i) sig.push_back(t_off[i]);
  for (const void* q : {(const void*)x, (const void*)out, (const void*)flags, (const void*)P.b_grid,
                        (const void*)P.b_far, (const void*)P.b_desc})
    sig.push_back((int64_t)(intptr_t)q);
  if (!P.b_exec || sig != P.b_sig) {
    free_batch(P);
    if (!P.b_capture) HIP_TRY(hipStreamCreateWithFlags(&P.b_capture, hipStreamNonBlocking));
    const bool timing = P.timing;
    P.timing = false;
    P.stream = P.b_capture;
    char* d = static_cast<char*>(P.b_desc);
    hipError_t e = hipStreamBeginCapture(P.b_capture, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) e = launch_fill2d_multi(P, d + Lo.fill_off, n_inst, Lo.fill_blocks, P.b_grid, spec);
    if (e == hipSuccess)
      e = launch_fft_multi(P, P.b_grid, reinterpret_cast<const FftSeg*>(d + Lo.segT_off), n_inst, Lo.segT_blocks,
                           Lo.lds_T);
    if (e == hipSuccess)
      e = launch_fft_multi(P, P.b_grid, reinterpret_cast<const FftSeg*>(d + Lo.segR_off), n_inst, Lo.segR_blocks,
                           Lo.lds_R);
    if (e == hipSuccess) e = launch_far2d_multi(P, d + Lo.far_off, n_inst, Lo.far_blocks, P.b_far);
    if (e == hipSuccess)
      e = launch_fft_multi(P, P.b_far, reinterpret_cast<const FftSeg*>(d + Lo.segF_off), n_inst, Lo.segF_blocks,
                           Lo.lds_F);
    if (e == hipSuccess && Lo.gat_blocks > 0)
      e = launch_gather2d_multi(P, d + Lo.gat_off, n_inst, Lo.gat_blocks, P.b_grid, P.b_far, x, out, flags);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(P.b_capture, &g);
    P.stream = user;
    P.timing = timing;
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&P.b_exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      P.b_exec = nullptr;
      return hip_fail(e, "batched graph capture");
    }
    P.b_graph = g;
    P.b_sig = sig;
  }
  KernelTimer t(P, QPGF_T_BATCH);
  HIP_TRY(hipGraphLaunch(P.b_exec, user));
  return QPGF_OK;
}

// ----------------------------------------------------------------------------
// FFT autotuner
// ----------------------------------------------------------------------------
extern "C" qpgf_status qpgf_plan_autotune(qpgf_plan* plan, const char* cache_path) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  Plan& P = plan->P;
  struct Shape { int n; bool rows; long batch; };
  std::vector<Shape> shapes;
  if (P.dim == 2) {
    shapes.push_back({P.M2, false, (long)P.M1 * P.nf});
    for (int n = 16; n <= P.M1; n <<= 1) shapes.push_back({n, true, (long)P.M2 * P.nf});
    if (P.M1 & (P.M1 - 1)) shapes.push_back({P.M1, true, (long)P.M2 * P.nf});   // 2^a r
    for (int n = 16; n <= P.Mf1; n <<= 1) shapes.push_back({n, true, (long)P.S * P.nfo});
  } else {
    shapes.push_back({P.M3, false, (long)P.M1 * P.M2 * P.nf});
    shapes.push_back({P.M2, false, (long)P.M1 * P.M3 * P.nf});
    shapes.push_back({P.M1, true, (long)P.M2 * P.M3 * P.nf});
    shapes.push_back({P.Mf2, false, (long)P.Mf1 * P.S * P.nfo});
    shapes.push_back({P.Mf1, true, (long)P.Mf2 * P.S * P.nfo});
  }
  const char* arch = "gfx950";
  const char* prec = P.p.prec == QPGF_C128 ? "c128" : "c64";
  std::map<std::string, int> cache;
  if (cache_path) {
    if (FILE* f = fopen(cache_path, "r")) {
      char a[32], pr[16], ax[8];
      int n, tile;
      long batch;
      double us;
      while (fscanf(f, "%31s %15s %d %7s %ld %d %lf", a, pr, &n, ax, &batch, &tile, &us) == 7)
        cache[std::string(a) + " " + pr + " " + std::to_string(n) + " " + ax + " " + std::to_string(batch)] = tile;
      fclose(f);
    }
  }
  size_t need = 0;
  for (const Shape& s : shapes) need = std::max(need, (size_t)s.n * s.batch * P.esize);
  void* tune_buf = nullptr;
  HIP_TRY(hipMalloc(&tune_buf, need));
  HIP_TRY(hipMemset(tune_buf, 0, need));
  hipEvent_t a = nullptr, b = nullptr;
  HIP_TRY(hipEventCreate(&a));
  HIP_TRY(hipEventCreate(&b));
  const bool timing = P.timing;
  P.timing = false;
  std::string lines;
  for (const Shape& s : shapes) {
    const std::string key = std::string(arch) + " " + prec + " " + std::to_string(s.n) + " " + (s.rows ? "rows" : "cols") +
                            " " + std::to_string(s.batch);
    const int mkey = (s.n << 2) | (s.rows ? 1 : 0) | (P.p.prec == QPGF_C64 ? 2 : 0);
    auto it = cache.find(key);
    if (it != cache.end()) {
      P.fft_tiles[mkey] = it->second;
      continue;
    }
    int best = 0;
    double best_us = 1e30;
    for (int tile = 1; tile <= 64; tile <<= 1) {
      if (tile > s.batch || (size_t)tile * (s.n + (s.rows ? 0 : 1)) * P.esize > 65536) break;
      P.fft_tiles[mkey] = tile;
      // rows: batches contiguous; cols: element stride = batch count, adjacent batches
      const long es = s.rows ? 1 : s.batch;
      const long b_in = s.rows ? 1 : s.batch, s_in = s.rows ? 0 : 1, s_out = s.rows ? s.n : 0;
      hipError_t e = hipSuccess;
      for (int w = 0; w < 2 && e == hipSuccess; ++w) e = launch_fft(P, tune_buf, s.n, es, s.batch, b_in, s_in, s_out);
      if (e == hipSuccess) e = hipEventRecord(a, P.stream);
      for (int r = 0; r < 5 && e == hipSuccess; ++r) e = launch_fft(P, tune_buf, s.n, es, s.batch, b_in, s_in, s_out);
      if (e == hipSuccess) e = hipEventRecord(b, P.stream);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (e != hipSuccess) {
        P.timing = timing;
        (void)hipFree(tune_buf);
        return hip_fail(e, "autotune");
      }
      const double us = 1000.0 * ms / 5;
      if (us < best_us) {
        best_us = us;
        best = tile;
      }
    }
    if (best > 0) {
      P.fft_tiles[mkey] = best;
      char buf[160];
      snprintf(buf, sizeof buf, "%s %s %d %s %ld %d %.3f\n", arch, prec, s.n, s.rows ? "rows" : "cols", s.batch, best,
               best_us);
      lines += buf;
    } else {
      P.fft_tiles.erase(mkey);
    }
  }
  P.timing = timing;
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  (void)hipFree(tune_buf);
  free_batch(P);   // a captured batched graph used the old tiles
  if (cache_path && !lines.empty()) {
    if (FILE* f = fopen(cache_path, "a")) {
      fputs(lines.c_str(), f);
      fclose(f);
    }
  }
  return QPGF_OK;
}

extern "C" {

qpgf_status qpgf_evaluate_smooth(qpgf_plan* plan, const double* x, int64_t T, void* out) {
  g_err.clear();
  qpgf_status st = check_plan(plan, QPGF_KIND_GD3D);
  if (st != QPGF_OK) return st;
  Plan& P = plan->P;
  if (T < 0) return fail(QPGF_E_ARG, "T < 0");
  if (T == 0) return QPGF_OK;
  if (!x || !out) return fail(QPGF_E_ARG, "x and out must be non-NULL device pointers");
  if (!P.prepared) return fail(QPGF_E_ARG, "evaluate before a complete prepare");
  if (T > (int64_t)0x7fffffff) return fail(QPGF_E_SIZE, "at most 2^31 - 1 targets per call");
  st = targets_fit(P, T);
  if (st != QPGF_OK) return st;
  HIP_TRY(launch_gather_smooth(P, x, T, out));
  return QPGF_OK;
}

qpgf_status qpgf_copy_field(qpgf_plan* plan, int which, int field, void* dst) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  Plan& P = plan->P;
  if (!dst) return fail(QPGF_E_ARG, "dst is NULL");
  if (which != 0 && which != 1) return fail(QPGF_E_ARG, "which must be 0 (near grid) or 1 (far slab)");
  if (field < 0 || field >= (which == 0 ? P.nf : P.nfo)) return fail(QPGF_E_ARG, "field out of range");
  const size_t n = (which == 0 ? P.ncell : P.nfar) * P.esize;
  const char* src = static_cast<const char*>(which == 0 ? P.grid : P.far) + (size_t)field * n;
  HIP_TRY(hipMemcpyAsync(dst, src, n, hipMemcpyDeviceToDevice, P.stream));
  return QPGF_OK;
}

qpgf_status qpgf_plan_enable_timing(qpgf_plan* plan, int on) {
  if (!plan) return fail(QPGF_E_ARG, "plan is NULL");
  drain_timers(plan->P);
  plan->P.timing = on != 0;
  for (int i = 0; i < QPGF_T_COUNT; ++i) {
    plan->P.t_ms[i] = 0.0;
    plan->P.t_n[i] = 0;
  }
  return QPGF_OK;
}

qpgf_status qpgf_plan_get_timing(qpgf_plan* plan, int id, double* total_ms, int64_t* launches) {
  if (!plan || !total_ms || !launches) return fail(QPGF_E_ARG, "plan, total_ms and launches must be non-NULL");
  if (id < 0 || id >= QPGF_T_COUNT) return fail(QPGF_E_ARG, "timer id out of range");
  drain_timers(plan->P);
  *total_ms = plan->P.t_ms[id];
  *launches = plan->P.t_n[id];
  return QPGF_OK;
}

const char* qpgf_last_error(void) { return g_err.c_str(); }

const char* qpgf_version(void) { return "qpgf 0.1 (gfx950)"; }

}  // extern "C"
