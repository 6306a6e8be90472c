// C ABI of libqpgf (include/qpgf.h): parameter validation, plan set-up
// (quadrature rules, twiddles, the 2D singular tables of Remark 2.1), the
// host-side exclusion checks (Wood anomalies, Section 1; the special
// coefficients of Sections 2.1 / 3.1) and the preparation / calculation
// sequences of Algorithms 2.1, 3.1 and 4.1.
#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>

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

void free_plan(Plan& P) {
  void* ptrs[] = {P.grid, P.far, P.xq,   P.wxq, P.cs,   P.rq,          P.wrq,  P.y1q,    P.y2q,    P.tw,
                  P.twf,  P.F1,  P.F2,   P.htab, P.bin_keyrank, P.bin_rec, P.bin_hist, P.bin_offs, P.bin_cnt, P.bin_ovf, P.bin_novf};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

qpgf_status validate(const qpgf_params* p) {
  if (!p) return fail(QPGF_E_ARG, "params is NULL");
  if (p->kind < 0 || p->kind > 2) return fail(QPGF_E_ARG, "unknown kind");
  if (p->prec != QPGF_C128 && p->prec != QPGF_C64) return fail(QPGF_E_ARG, "unknown precision");
  if (!pow2_in(p->m1, 16, 4096) || !pow2_in(p->m2, 16, 4096))
    return fail(QPGF_E_SIZE, "m1 and m2 must be powers of two in [16, 4096]");
  if (p->kind != QPGF_KIND_G2D && !pow2_in(p->m3, 16, 4096))
    return fail(QPGF_E_SIZE, "m3 must be a power of two in [16, 4096]");
  if (!(p->c > 0.0) || !(p->c_tilde > p->c)) return fail(QPGF_E_ARG, "need 0 < c < c_tilde");
  if (!(p->eps > 0.0) || !(2.0 * p->eps <= p->c_tilde)) return fail(QPGF_E_ARG, "need 0 < 2 eps <= c_tilde");
  if (p->quad_q < 16 || p->quad_q > 256) return fail(QPGF_E_ARG, "quad_q must be in [16, 256]");
  if (!(p->far_h > 0.0) || !(p->far_zmax >= p->c)) return fail(QPGF_E_ARG, "need far_h > 0 and far_zmax >= c");
  if (!(p->wood_tol >= 0.0) || !(p->special_tol >= 0.0) || !(p->lattice_rmin >= 0.0))
    return fail(QPGF_E_ARG, "tolerances must be >= 0");
  return QPGF_OK;
}

// Wood anomaly: beta_n = 0 for some mode n (Section 1).  Only lattice points with
// |xi_perp| within 1 of k can come close.
qpgf_status check_instance(const Plan& P, double k, double a1, double a2) {
  if (!(k > 0.0) || !std::isfinite(k) || !std::isfinite(a1) || !std::isfinite(a2))
    return fail(QPGF_E_ARG, "need finite k > 0 and finite alpha");
  const double wt = P.p.wood_tol, st = P.p.special_tol;
  const int Nt = P.Mt / 2;
  auto special = [&](double rho) -> bool {
    // |beta - |J|| for a propagating beta against every transverse index of the grid
    if (rho >= k) return false;
    double b = sqrt((k - rho) * (k + rho));
    double jt = std::round(b * P.p.c_tilde / M_PI);
    if (jt > Nt) return false;
    return fabs(b - jt * M_PI / P.p.c_tilde) < st;
  };
  double minb = 1e300;
  if (P.dim == 2) {
    for (long n = (long)floor(-k - a1) - 1; n <= (long)ceil(k - a1) + 1; ++n) {
      double rho = fabs(a1 + n);
      minb = std::min(minb, sqrt(fabs((k - rho) * (k + rho))));
      if (n >= -P.M1 / 2 && n < P.M1 / 2 && special(rho))
        return fail(QPGF_E_SPECIAL, "beta_j1 = j2 pi / c_tilde within special_tol (perturb c_tilde)");
    }
  } else {
    for (long n1 = (long)floor(-k - a1) - 1; n1 <= (long)ceil(k - a1) + 1; ++n1)
      for (long n2 = (long)floor(-k - a2) - 1; n2 <= (long)ceil(k - a2) + 1; ++n2) {
        double rho = sqrt((a1 + n1) * (a1 + n1) + (a2 + n2) * (a2 + n2));
        minb = std::min(minb, sqrt(fabs((k - rho) * (k + rho))));
        if (n1 >= -P.M1 / 2 && n1 < P.M1 / 2 && n2 >= -P.M2 / 2 && n2 < P.M2 / 2 && special(rho))
          return fail(QPGF_E_SPECIAL, "beta_j1j2 = j3 pi / c_tilde within special_tol (perturb c_tilde)");
      }
  }
  if (minb < wt) {
    char buf[160];
    snprintf(buf, sizeof buf, "Wood anomaly: min |beta| = %.3e < wood_tol = %.3e", minb, wt);
    return fail(QPGF_E_WOOD, buf);
  }
  return QPGF_OK;
}

qpgf_status run_prepare(Plan& P, double k, double a1, double a2, int stage) {
  qpgf_status st = check_instance(P, k, a1, a2);
  if (st != QPGF_OK) return st;
  P.last_k = k;
  P.last_a1 = a1;
  P.last_a2 = a2;
  P.prepared = false;
  if (P.dim == 3) {
    // H table must cover |xi| over the grid's modes
    const double e1 = P.M1 / 2 + fabs(a1) + 1.0, e2 = P.M2 / 2 + fabs(a2) + 1.0;
    const double e3 = (P.M3 / 2 + 1.0) * M_PI / P.p.c_tilde;
    const int need = (int)(sqrt(e1 * e1 + e2 * e2 + e3 * e3) / P.hd) + 16;
    if (need > P.hn) {
      if (P.htab) HIP_TRY(hipFree(P.htab));
      P.htab = nullptr;
      HIP_TRY(hipMalloc(reinterpret_cast<void**>(&P.htab), (size_t)need * sizeof(double2)));
      P.hn = need;
    }
    KernelTimer t(P, QPGF_T_HTABLE);
    HIP_TRY(launch_htable(P, k));
  }
  {
    KernelTimer t(P, QPGF_T_FILL);
    HIP_TRY(launch_fill(P, k, a1, a2));
  }
  if (stage >= 1) {
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
      KernelTimer t(P, QPGF_T_FAR_FFT);
      if (P.dim == 3)
        HIP_TRY(launch_fft(P, P.far, P.M2, P.M1, (long)P.M1 * P.S * nf, P.M1, 1, (long)P.M1 * P.M2));
      HIP_TRY(launch_fft(P, P.far, P.M1, 1, (long)(P.dim == 3 ? P.M2 : 1) * P.S * nf, 1, 0, P.M1));
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
  HIP_TRY(launch_gather(P, x, T, out, flags));
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
  const int mt = (kind == QPGF_KIND_G2D) ? m2 : m3;
  p->far_h = mt > 0 ? p->c_tilde / (mt / 2) : 0.0;
  p->far_zmax = p->c_tilde;
  p->wood_tol = 1e-3;
  p->special_tol = 1e-6;
  p->lattice_rmin = 0.0;
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
  P.dim = (p->kind == QPGF_KIND_G2D) ? 2 : 3;
  P.nf = (p->kind == QPGF_KIND_MAXWELL3D) ? 7 : 1;
  P.M1 = p->m1;
  P.M2 = p->m2;
  P.M3 = (P.dim == 3) ? p->m3 : 1;
  P.Mt = (P.dim == 3) ? P.M3 : P.M2;
  P.esize = (p->prec == QPGF_C128) ? 16 : 8;
  P.S = (int)std::ceil((p->far_zmax - p->c) / p->far_h - 1e-12) + 4;
  P.ncell = (size_t)P.M1 * P.M2 * P.M3;
  P.nfar = (size_t)P.M1 * (P.dim == 3 ? P.M2 : 1) * P.S;

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

  PLAN_TRY(hipMalloc(&P.grid, P.nf * P.ncell * P.esize));
  PLAN_TRY(hipMalloc(&P.far, P.nf * P.nfar * P.esize));

  const int Q = p->quad_q;
  std::vector<long double> gx, gw;
  gauss_legendre(Q, gx, gw);
  // X'-integral rule on [c, (c + c~)/2]: X'(x) = -S'((x - c)/w)/w, w = (c~ - c)/2
  {
    const long double c = p->c, w = 0.5L * (p->c_tilde - p->c);
    std::vector<double> xq(Q), wxq(Q);
    for (int q = 0; q < Q; ++q) {
      long double x = c + 0.5L * w * (gx[q] + 1.0L);
      long double u = (x - c) / w;
      xq[q] = (double)x;
      wxq[q] = (double)(0.5L * w * gw[q] * (-(long double)smooth_S1((double)u) / w));
    }
    PLAN_ST(upload(&P.xq, xq));
    PLAN_ST(upload(&P.wxq, wxq));
    const int Nt = P.Mt / 2;
    std::vector<double2> cs((size_t)(Nt + 1) * Q);
    for (int j = 0; j <= Nt; ++j)
      for (int q = 0; q < Q; ++q) {
        long double a = (long double)j * kPiL / p->c_tilde * (long double)xq[q];
        cs[(size_t)j * Q + q] = make_double2((double)cosl(a), (double)sinl(a));
      }
    PLAN_ST(upload(&P.cs, cs));
  }
  // radial rule on [eps, 2 eps] with Y', Y'' at the nodes
  std::vector<double> rq(Q), wrq(Q), y1q(Q), y2q(Q);
  {
    const long double e = p->eps;
    for (int q = 0; q < Q; ++q) {
      long double r = e + 0.5L * e * (gx[q] + 1.0L);
      rq[q] = (double)r;
      wrq[q] = (double)(0.5L * e * gw[q]);
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
    int NT = std::max(P.M1, std::max(P.M2, P.M3));
    P.twlog2 = __builtin_ctz((unsigned)NT);
    std::vector<double2> tw(NT);
    std::vector<float2> twf(NT);
    for (int j = 0; j < NT; ++j) {
      long double a = 2.0L * kPiL * j / NT;
      tw[j] = make_double2((double)cosl(a), (double)sinl(a));
      twf[j] = make_float2((float)cosl(a), (float)sinl(a));
    }
    PLAN_ST(upload(&P.tw, tw));
    PLAN_ST(upload(&P.twf, twf));
  }
  if (P.dim == 2) {
    // Phi_1(r) = (2 + ln r) Y'(r)/r + Y''(r) ln r at the radial nodes, times the weights
    std::vector<double> wphi(Q);
    long double f1tail = 0.0L;
    for (int q = 0; q < Q; ++q) {
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
  info->far_h = P.p.far_h;
  info->c = P.p.c;
  info->c_tilde = P.p.c_tilde;
  info->eps = P.p.eps;
  info->n_fields = P.nf;
  info->grid_bytes = P.ncell * P.esize;
  info->far_grid_bytes = P.nfar * P.esize;
  return QPGF_OK;
}

qpgf_status qpgf_prepare(qpgf_plan* plan, double k, double a1, double a2) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  return run_prepare(plan->P, k, a1, plan->P.dim == 3 ? a2 : 0.0, 2);
}

qpgf_status qpgf_prepare_stage(qpgf_plan* plan, double k, double a1, double a2, int stage) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  if (stage < 0 || stage > 2) return fail(QPGF_E_ARG, "stage must be 0, 1 or 2");
  return run_prepare(plan->P, k, a1, plan->P.dim == 3 ? a2 : 0.0, stage);
}

qpgf_status qpgf_evaluate(qpgf_plan* plan, const double* x, int64_t T, void* out, uint8_t* flags) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  return run_evaluate(plan->P, x, T, out, flags);
}

static qpgf_status both(qpgf_plan* plan, int kind, double k, double a1, double a2, const double* x, int64_t T,
                        void* out, uint8_t* flags) {
  g_err.clear();
  qpgf_status st = check_plan(plan, kind);
  if (st != QPGF_OK) return st;
  if (T < 0) return fail(QPGF_E_ARG, "T < 0");
  if (T > 0 && (!x || !out)) return fail(QPGF_E_ARG, "x and out must be non-NULL device pointers");
  st = run_prepare(plan->P, k, a1, a2, 2);
  if (st != QPGF_OK) return st;
  return run_evaluate(plan->P, x, T, out, flags);
}

qpgf_status qpgf_g2d(qpgf_plan* plan, double k, double alpha, const double* x, int64_t T, void* out,
                     uint8_t* flags) {
  return both(plan, QPGF_KIND_G2D, k, alpha, 0.0, x, T, out, flags);
}

qpgf_status qpgf_gd3d(qpgf_plan* plan, double k, double a1, double a2, const double* x, int64_t T, void* out,
                      uint8_t* flags) {
  return both(plan, QPGF_KIND_GD3D, k, a1, a2, x, T, out, flags);
}

qpgf_status qpgf_maxwell3d(qpgf_plan* plan, double k, double a1, double a2, const double* x, int64_t T,
                           void* out, uint8_t* flags) {
  return both(plan, QPGF_KIND_MAXWELL3D, k, a1, a2, x, T, out, flags);
}

qpgf_status qpgf_copy_field(qpgf_plan* plan, int which, int field, void* dst) {
  g_err.clear();
  qpgf_status st = check_plan(plan, -1);
  if (st != QPGF_OK) return st;
  Plan& P = plan->P;
  if (!dst) return fail(QPGF_E_ARG, "dst is NULL");
  if (which != 0 && which != 1) return fail(QPGF_E_ARG, "which must be 0 (near grid) or 1 (far slab)");
  if (field < 0 || field >= P.nf) return fail(QPGF_E_ARG, "field out of range");
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
