// C ABI of the MLP surrogate: model state, training step (forward, backward,
// Adam), inference for many instances with fallback to the plain method.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "qpgf_internal.h"

namespace qpgf {
hipError_t mlp_gemm(hipStream_t st, const __bf16* A, long a_m, long a_k, const __bf16* B, long b_k, long b_n,
                    float* C, long c_m, long c_n, const float* bias, int M, int N, int K, int splits);
hipError_t mlp_gelu_fwd(hipStream_t st, const float* Z, long M, int N, __bf16* A, __bf16* AT);
hipError_t mlp_gelu_bwd(hipStream_t st, const float* dA, const float* Z, long M, int N, __bf16* dZ, __bf16* dZT,
                        float* dZf);
hipError_t mlp_sum_parts(hipStream_t st, const float* p, int parts, long n, float* out);
hipError_t mlp_colsum(hipStream_t st, const float* X, long M, int N, float* out);
hipError_t mlp_head_fwd(hipStream_t st, const __bf16* A, const float* W, const float* b, long M, float* out);
hipError_t mlp_head_bwd(hipStream_t st, const __bf16* A, const float* W, const float* out, const float* y, long M,
                        float* dA, float* part);
hipError_t mlp_adam(hipStream_t st, float* p, const float* g, float* m1, float* m2, long n, float lr, float b1,
                    float b2, float eps, float c1, float c2);
hipError_t mlp_refresh_bf16(hipStream_t st, const float* W, int N, int K, __bf16* Wb, __bf16* WTb);
hipError_t mlp_features(hipStream_t st, const double* q, long M, double c, double c_tilde, __bf16* F, __bf16* FT);
size_t mlp_qinst_size();
size_t mlp_qinst_t0_offset();
void mlp_qinst(double k, double a1, double a2, long t0, long t1, void* dst);
hipError_t mlp_make_queries(hipStream_t st, const void* inst, int n, const double* x, long T, double* q);
hipError_t mlp_combine(hipStream_t st, int prec, const double* q, long M, const float* y, int members, long ystride,
                       double c, double eps, double tol, double kappa, double wood_tol, double rmin, void* out,
                       uint8_t* fell);
hipError_t mlp_calib_ratio(hipStream_t st, int prec, long M, const float* y, int members, long ystride, const void* L,
                           double* ratio);
hipError_t mlp_make_rows(hipStream_t st, int prec, const double* x, long n, double k, double a1, double a2,
                         const void* L, double* q, float* y);
hipError_t mlp_gather_rows(hipStream_t st, const double* q, const float* y, const uint32_t* idx, long B, double* qb,
                           float* yb);
hipError_t launch_gather_smooth(Plan& P, const double* x, int64_t T, void* out);
hipError_t mlp_infer(hipStream_t st, const __bf16* const* wb, const float* const* p, int members, const long off_b[4],
                     long off_w4, long off_b4, double c, double c_tilde, const double* q, long M, float* y,
                     long ystride);
}  // namespace qpgf

using namespace qpgf;

namespace {

thread_local std::string s_err;
constexpr int D_IN = 64, H = 256, NOUT = 2;
constexpr double kC = 0.6, kCt = 1.0;   // near region |x3| <= c and x3 period 2 c~ of the modelled L_d
// flat parameter layout of one member
constexpr long OFF_W0 = 0, OFF_B0 = OFF_W0 + (long)H * D_IN;
constexpr long OFF_W1 = OFF_B0 + H, OFF_B1 = OFF_W1 + (long)H * H;
constexpr long OFF_W2 = OFF_B1 + H, OFF_B2 = OFF_W2 + (long)H * H;
constexpr long OFF_W3 = OFF_B2 + H, OFF_B3 = OFF_W3 + (long)H * H;
constexpr long OFF_W4 = OFF_B3 + H, OFF_B4 = OFF_W4 + (long)NOUT * H;
constexpr long NPARAM = OFF_B4 + NOUT;
constexpr long W_OFF[4] = {OFF_W0, OFF_W1, OFF_W2, OFF_W3};
constexpr long B_OFF[4] = {OFF_B0, OFF_B1, OFF_B2, OFF_B3};
constexpr int K_IN[4] = {D_IN, H, H, H};

}  // namespace

struct qpgf_mlp {
  int members = 1;
  long maxb = 0;                 // rows per pass (multiple of 64)
  hipStream_t stream = nullptr;
  // per member
  std::vector<float*> p, m1, m2; // fp32 params and Adam moments [NPARAM]
  std::vector<__bf16*> wb;       // bf16 hidden weights, 4 matrices back to back
  std::vector<long> step;
  double kappa = HUGE_VAL;       // error-estimate calibration: |L_mean - L| <= kappa * spread; +inf = none
  // work buffers (maxb rows)
  double* q = nullptr;           // training minibatch queries [maxb][6]
  __bf16 *F = nullptr, *FT = nullptr;
  float* Z[4] = {};              // pre-activations [maxb][H]
  __bf16* A[4] = {};             // activations [maxb][H]
  float* out = nullptr;          // [maxb][2]
  float *dA = nullptr, *dZf = nullptr;
  __bf16 *dZ = nullptr, *dZT = nullptr;
  float* part = nullptr;         // split / block partial sums
  float* grad = nullptr;         // [NPARAM]
  float* ybuf = nullptr;         // ensemble outputs [members][maxb][2]
  // fallback scratch
  uint32_t* counts = nullptr;
  uint32_t* cursor = nullptr;
  uint32_t* fidx = nullptr;
  size_t fidx_cap = 0;
  double* fx = nullptr;
  void* fout = nullptr;
  size_t fx_cap = 0;
  void* qinst = nullptr;
  size_t qinst_cap = 0;
  double* qall = nullptr;
  size_t qall_cap = 0;
  uint32_t* perm = nullptr;      // training data order [perm_cap]
  size_t perm_cap = 0;
};

namespace {

qpgf_status sfail(qpgf_status s, const std::string& m) {
  s_err = m;
  return s;
}
#define S_TRY(call)                                                                                      \
  do {                                                                                                   \
    hipError_t e_ = (call);                                                                              \
    if (e_ != hipSuccess)                                                                                \
      return sfail(e_ == hipErrorOutOfMemory ? QPGF_E_NOMEM : QPGF_E_HIP, std::string(#call) + ": " +   \
                   hipGetErrorString(e_));                                                               \
  } while (0)

template <typename V>
hipError_t dalloc(V** p, size_t n) {
  return hipMalloc(reinterpret_cast<void**>(p), n * sizeof(V));
}

uint64_t splitmix(uint64_t& s) {
  uint64_t z = (s += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

hipError_t refresh(qpgf_mlp* m, int e) {
  for (int l = 0; l < 4; ++l) {
    hipError_t r = mlp_refresh_bf16(m->stream, m->p[e] + W_OFF[l], H, K_IN[l], m->wb[e] + (long)l * H * H, nullptr);
    if (r != hipSuccess) return r;
  }
  return hipSuccess;
}

// forward pass of member e on rows [0, Mp) of features m->F (Mp multiple of 64)
hipError_t forward(qpgf_mlp* m, int e, long Mp, float* out) {
  hipError_t r = hipSuccess;
  const __bf16* X = m->F;
  long ldx = D_IN;
  for (int l = 0; l < 4 && r == hipSuccess; ++l) {
    const __bf16* W = m->wb[e] + (long)l * H * H;
    r = mlp_gemm(m->stream, X, ldx, 1, W, 1, K_IN[l], m->Z[l], H, 1, m->p[e] + B_OFF[l], (int)Mp, H, K_IN[l], 1);
    if (r == hipSuccess) r = mlp_gelu_fwd(m->stream, m->Z[l], Mp, H, m->A[l], nullptr);
    X = m->A[l];
    ldx = H;
  }
  if (r == hipSuccess) r = mlp_head_fwd(m->stream, m->A[3], m->p[e] + OFF_W4, m->p[e] + OFF_B4, Mp, out);
  return r;
}

// gradient of 0.5 mean |out - y|^2 over rows [0, Mp) into m->grad; loss into part[.]
hipError_t backward(qpgf_mlp* m, int e, long Mp, const float* y, float* loss) {
  hipError_t r = hipSuccess;
  const long nblk = (Mp + 255) / 256;
  r = mlp_head_bwd(m->stream, m->A[3], m->p[e] + OFF_W4, m->out, y, Mp, m->dA, m->part);
  // reduce per-block [loss, db0, db1, dW4 (512)] partials
  float* red = m->part + nblk * 515;
  if (r == hipSuccess) r = mlp_sum_parts(m->stream, m->part, (int)nblk, 515, red);
  if (r == hipSuccess && loss) r = hipMemcpyAsync(loss, red, sizeof(float), hipMemcpyDeviceToDevice, m->stream);
  if (r == hipSuccess)
    r = hipMemcpyAsync(m->grad + OFF_B4, red + 1, 2 * sizeof(float), hipMemcpyDeviceToDevice, m->stream);
  if (r == hipSuccess)
    r = hipMemcpyAsync(m->grad + OFF_W4, red + 3, 512 * sizeof(float), hipMemcpyDeviceToDevice, m->stream);
  for (int l = 3; l >= 0 && r == hipSuccess; --l) {
    r = mlp_gelu_bwd(m->stream, m->dA, m->Z[l], Mp, H, m->dZ, m->dZT, m->dZf);
    const __bf16* Xin = l == 0 ? m->F : m->A[l - 1];
    const int K = K_IN[l];
    // dW_l [H x K] = dZ^T X_in, split over the batch
    const int splits = (int)std::max(1L, std::min(32L, Mp / 512));
    if (r == hipSuccess)
      r = mlp_gemm(m->stream, m->dZT, Mp, 1, Xin, K, 1, m->part, K, 1, nullptr, H, K, (int)Mp, splits);
    if (r == hipSuccess) r = mlp_sum_parts(m->stream, m->part, splits, (long)H * K, m->grad + W_OFF[l]);
    if (r == hipSuccess) r = mlp_colsum(m->stream, m->dZf, Mp, H, m->grad + B_OFF[l]);
    // dX_{l-1} = dZ W_l (fp32), not needed for the input features
    if (l > 0 && r == hipSuccess)
      r = mlp_gemm(m->stream, m->dZ, H, 1, m->wb[e] + (long)l * H * H, K, 1, m->dA, K, 1, nullptr, (int)Mp, K, H, 1);
  }
  return r;
}

qpgf_status check_mlp(const qpgf_mlp* m, int e) {
  if (!m) return sfail(QPGF_E_ARG, "model is NULL");
  if (e < 0 || e >= m->members) return sfail(QPGF_E_ARG, "member out of range");
  return QPGF_OK;
}

}  // namespace

extern "C" {

long qpgf_mlp_param_count(void) { return NPARAM; }

qpgf_status qpgf_mlp_create(int members, int64_t max_batch, uint64_t seed, qpgf_mlp** out) {
  s_err.clear();
  if (!out) return sfail(QPGF_E_ARG, "out is NULL");
  *out = nullptr;
  if (members < 1 || members > 8) return sfail(QPGF_E_ARG, "members must be in [1, 8]");
  if (max_batch < 64 || max_batch % 64 || max_batch > (1 << 22))
    return sfail(QPGF_E_ARG, "max_batch must be a multiple of 64 in [64, 2^22]");
  auto* m = new (std::nothrow) qpgf_mlp();
  if (!m) return sfail(QPGF_E_NOMEM, "host allocation");
  m->members = members;
  m->maxb = max_batch;
  const long B = max_batch;
  auto bail = [&](hipError_t e) {
    s_err = std::string("allocation: ") + hipGetErrorString(e);
    qpgf_mlp_destroy(m);
    return e == hipErrorOutOfMemory ? QPGF_E_NOMEM : QPGF_E_HIP;
  };
  hipError_t e = hipSuccess;
  std::vector<float> host(NPARAM);
  for (int k = 0; k < members && e == hipSuccess; ++k) {
    float *p = nullptr, *a = nullptr, *b = nullptr;
    __bf16* w = nullptr;
    e = dalloc(&p, NPARAM);
    if (e == hipSuccess) e = dalloc(&a, NPARAM);
    if (e == hipSuccess) e = dalloc(&b, NPARAM);
    if (e == hipSuccess) e = dalloc(&w, (size_t)4 * H * H);
    m->p.push_back(p);
    m->m1.push_back(a);
    m->m2.push_back(b);
    m->wb.push_back(w);
    m->step.push_back(0);
    if (e != hipSuccess) break;
    // He-uniform hidden weights, small head, zero biases; one stream of draws per member
    uint64_t s = seed * 1000003ull + 7919ull * (uint64_t)k + 1ull;
    std::fill(host.begin(), host.end(), 0.f);
    for (int l = 0; l < 4; ++l) {
      const float bound = sqrtf(6.f / K_IN[l]);
      for (long i = 0; i < (long)H * K_IN[l]; ++i)
        host[W_OFF[l] + i] = bound * (2.f * (float)((splitmix(s) >> 11) * 0x1.0p-53) - 1.f);
    }
    for (long i = 0; i < (long)NOUT * H; ++i)
      host[OFF_W4 + i] = sqrtf(1.f / H) * (2.f * (float)((splitmix(s) >> 11) * 0x1.0p-53) - 1.f);
    e = hipMemcpy(p, host.data(), NPARAM * sizeof(float), hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemset(a, 0, NPARAM * sizeof(float));
    if (e == hipSuccess) e = hipMemset(b, 0, NPARAM * sizeof(float));
  }
  if (e == hipSuccess) e = dalloc(&m->F, (size_t)B * D_IN);
  if (e == hipSuccess) e = dalloc(&m->FT, (size_t)B * D_IN);
  for (int l = 0; l < 4 && e == hipSuccess; ++l) {
    e = dalloc(&m->Z[l], (size_t)B * H);
    if (e == hipSuccess) e = dalloc(&m->A[l], (size_t)B * H);
  }
  if (e == hipSuccess) e = dalloc(&m->out, (size_t)B * NOUT);
  if (e == hipSuccess) e = dalloc(&m->dA, (size_t)B * H);
  if (e == hipSuccess) e = dalloc(&m->dZf, (size_t)B * H);
  if (e == hipSuccess) e = dalloc(&m->dZ, (size_t)B * H);
  if (e == hipSuccess) e = dalloc(&m->dZT, std::max((size_t)B * H, (size_t)H * H));
  // partials: split-K GEMM (32 x H x H) or head blocks (B/256 x 515) plus the reduced row
  if (e == hipSuccess) e = dalloc(&m->part, std::max((size_t)32 * H * H, (size_t)(B / 256 + 2) * 515));
  if (e == hipSuccess) e = dalloc(&m->grad, (size_t)NPARAM);
  if (e == hipSuccess) e = dalloc(&m->ybuf, (size_t)members * B * NOUT);
  if (e == hipSuccess) e = dalloc(&m->q, (size_t)B * 6);
  if (e != hipSuccess) return bail(e);
  for (int k = 0; k < members; ++k) {
    e = refresh(m, k);
    if (e != hipSuccess) return bail(e);
  }
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return bail(e);
  *out = m;
  return QPGF_OK;
}

void qpgf_mlp_destroy(qpgf_mlp* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  for (auto* v : m->p) if (v) (void)hipFree(v);
  for (auto* v : m->m1) if (v) (void)hipFree(v);
  for (auto* v : m->m2) if (v) (void)hipFree(v);
  for (auto* v : m->wb) if (v) (void)hipFree(v);
  void* ptrs[] = {m->q, m->F, m->FT, m->out, m->dA, m->dZf, m->dZ, m->dZT, m->part, m->grad, m->ybuf, m->counts,
                  m->cursor, m->fidx, m->fx, m->fout, m->qinst, m->qall, m->perm};
  for (void* v : ptrs)
    if (v) (void)hipFree(v);
  for (int l = 0; l < 4; ++l) {
    if (m->Z[l]) (void)hipFree(m->Z[l]);
    if (m->A[l]) (void)hipFree(m->A[l]);
  }
  delete m;
}

qpgf_status qpgf_mlp_set_stream(qpgf_mlp* m, void* stream) {
  if (!m) return sfail(QPGF_E_ARG, "model is NULL");
  m->stream = static_cast<hipStream_t>(stream);
  return QPGF_OK;
}

qpgf_status qpgf_mlp_get_params(qpgf_mlp* m, int member, float* dst) {
  qpgf_status st = check_mlp(m, member);
  if (st != QPGF_OK) return st;
  if (!dst) return sfail(QPGF_E_ARG, "dst is NULL");
  S_TRY(hipMemcpyAsync(dst, m->p[member], NPARAM * sizeof(float), hipMemcpyDeviceToDevice, m->stream));
  return QPGF_OK;
}

qpgf_status qpgf_mlp_set_params(qpgf_mlp* m, int member, const float* src) {
  qpgf_status st = check_mlp(m, member);
  if (st != QPGF_OK) return st;
  if (!src) return sfail(QPGF_E_ARG, "src is NULL");
  S_TRY(hipMemcpyAsync(m->p[member], src, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, m->stream));
  S_TRY(refresh(m, member));
  return QPGF_OK;
}

// y[B][2] = network(q[B][6]) for member e; B any size (internally padded to 64).
qpgf_status qpgf_mlp_forward(qpgf_mlp* m, int member, const double* q, int64_t B, float* y) {
  s_err.clear();
  qpgf_status st = check_mlp(m, member);
  if (st != QPGF_OK) return st;
  if (B < 0 || (B > 0 && (!q || !y))) return sfail(QPGF_E_ARG, "bad arguments");
  if (B == 0) return QPGF_OK;
  // the fused inference kernel: no intermediate buffers, any B
  const __bf16* wb[1] = {m->wb[member]};
  const float* pp[1] = {m->p[member]};
  S_TRY(mlp_infer(m->stream, wb, pp, 1, B_OFF, OFF_W4, OFF_B4, kC, kCt, q, (long)B, y, 0));
  return QPGF_OK;
}

// Gradient (flat, [NPARAM]) of 0.5 mean_b |net(q_b) - y_b|^2 for member e; B a multiple of 64, <= max_batch.
qpgf_status qpgf_mlp_gradient(qpgf_mlp* m, int member, const double* q, const float* y, int64_t B, float* grad,
                              float* loss) {
  s_err.clear();
  qpgf_status st = check_mlp(m, member);
  if (st != QPGF_OK) return st;
  if (B < 64 || B % 64 || B > m->maxb || !q || !y) return sfail(QPGF_E_ARG, "B must be a multiple of 64 <= max_batch");
  S_TRY(mlp_features(m->stream, q, B, kC, kCt, m->F, nullptr));
  S_TRY(forward(m, member, B, m->out));
  S_TRY(backward(m, member, B, y, loss));
  if (grad) S_TRY(hipMemcpyAsync(grad, m->grad, NPARAM * sizeof(float), hipMemcpyDeviceToDevice, m->stream));
  return QPGF_OK;
}

qpgf_status qpgf_mlp_train_step(qpgf_mlp* m, int member, const double* q, const float* y, int64_t B, float lr,
                                float* loss) {
  qpgf_status st = qpgf_mlp_gradient(m, member, q, y, B, nullptr, loss);
  if (st != QPGF_OK) return st;
  const float b1 = 0.9f, b2 = 0.999f;
  const long t = ++m->step[member];
  const float c1 = 1.f - powf(b1, (float)t), c2 = 1.f - powf(b2, (float)t);
  S_TRY(mlp_adam(m->stream, m->p[member], m->grad, m->m1[member], m->m2[member], NPARAM, lr, b1, b2, 1e-8f, c1, c2));
  S_TRY(refresh(m, member));
  return QPGF_OK;
}

const char* qpgf_mlp_last_error(void) { return s_err.c_str(); }

}  // extern "C"

// ---------------------------------------------------------------------------
// Surrogate evaluation with fallback
// ---------------------------------------------------------------------------
namespace {

// Targets of one instance are contiguous, so the lanes of a wave that belong to the same
// instance form one run of lanes; each run adds its fallback count with one atomic (one atomic
// per target on a single counter per instance serialises the whole pass).
__global__ void k_count_fallback(const uint8_t* __restrict__ fell, const void* __restrict__ qinst, int n_inst,
                                 size_t isz, size_t t0off, long T, uint32_t* __restrict__ counts,
                                 uint32_t* __restrict__ cursor, const uint32_t* __restrict__ offs,
                                 uint32_t* __restrict__ fidx, int pass) {
  const long m = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool in = m < T;
  const bool f = in && fell[m];
  int lo = n_inst;  // lanes past the end form a run of their own that counts nothing
  if (in) {
    // instance of target m: binary search on the instances' first target
    int l = 0, hi = n_inst - 1;
    const char* base = static_cast<const char*>(qinst);
    while (l < hi) {
      const int mid = (l + hi + 1) >> 1;
      const long t0 = *reinterpret_cast<const long*>(base + mid * isz + t0off);
      if (t0 <= m) l = mid;
      else hi = mid - 1;
    }
    lo = l;
  }
  const int lane = __lane_id();
  const int prev = __shfl_up(lo, 1);
  const unsigned long long H = __ballot(lane == 0 || prev != lo);  // first lane of each run
  const unsigned long long F = __ballot(f);
  const unsigned long long upto = (2ull << lane) - 1;  // lanes 0..lane
  const int s = 63 - __clzll(H & upto);
  const unsigned long long after = H & ~upto;
  const int e = after ? __ffsll((long long)after) - 1 : 64;
  const unsigned long long run = (e == 64 ? ~0ull : ((1ull << e) - 1)) & ~((1ull << s) - 1);
  const unsigned n = (unsigned)__popcll(F & run);
  unsigned first = 0;
  if (lane == s && n && lo < n_inst) {
    if (pass == 0) atomicAdd(&counts[lo], n);
    else first = atomicAdd(&cursor[lo], n);
  }
  first = __shfl(first, s);
  if (pass == 1 && f) fidx[offs[lo] + first + (unsigned)__popcll(F & run & ((1ull << lane) - 1))] = (uint32_t)m;
}

__global__ void k_pick(const double* __restrict__ x, const uint32_t* __restrict__ idx, long n, double* __restrict__ y) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long m = idx[i];
  y[3 * i] = x[3 * m];
  y[3 * i + 1] = x[3 * m + 1];
  y[3 * i + 2] = x[3 * m + 2];
}

__global__ void k_put(const char* __restrict__ src, const uint32_t* __restrict__ idx, long n, size_t esize,
                      char* __restrict__ dst) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const long m = idx[i];
  for (size_t b = 0; b < esize; ++b) dst[m * esize + b] = src[i * esize + b];
}

unsigned gb(long n) { return (unsigned)((n + 255) / 256); }

}  // namespace

extern "C" qpgf_status qpgf_surrogate_eval(qpgf_mlp* m, qpgf_plan* plan, double tol, double wood_tol, double rmin,
                                           int n_inst, const double* k, const double* a1, const double* a2,
                                           const int64_t* t_off, const double* x, void* out, uint8_t* fell_back,
                                           int64_t* n_fallback);

qpgf_status qpgf_surrogate_eval(qpgf_mlp* m, qpgf_plan* plan, double tol, double wood_tol, double rmin, int n_inst,
                                const double* k, const double* a1, const double* a2, const int64_t* t_off,
                                const double* x, void* out, uint8_t* fell_back, int64_t* n_fallback) {
  s_err.clear();
  if (!m || !plan) return sfail(QPGF_E_ARG, "model and plan must be non-NULL");
  qpgf_plan_info info;
  if (qpgf_plan_get_info(plan, &info) != QPGF_OK || info.kind != QPGF_KIND_GD3D)
    return sfail(QPGF_E_ARG, "the fallback plan must be of kind GD3D");
  if (info.c != kC || info.c_tilde != kCt)
    return sfail(QPGF_E_ARG, "the fallback plan must use the surrogate's c = 0.6 and c_tilde = 1");
  if (n_inst <= 0 || !k || !a1 || !a2 || !t_off || !fell_back) return sfail(QPGF_E_ARG, "bad instance arguments");
  const int64_t T = t_off[n_inst];
  if (T <= 0) return QPGF_OK;
  if (!x || !out) return sfail(QPGF_E_ARG, "x and out must be non-NULL");
  const size_t isz = mlp_qinst_size();
  if ((size_t)n_inst * isz > m->qinst_cap) {
    if (m->qinst) (void)hipFree(m->qinst);
    m->qinst = nullptr;
    S_TRY(hipMalloc(&m->qinst, (size_t)n_inst * isz));
    m->qinst_cap = (size_t)n_inst * isz;
    if (m->counts) (void)hipFree(m->counts);
    if (m->cursor) (void)hipFree(m->cursor);
    m->counts = m->cursor = nullptr;
    S_TRY(dalloc(&m->counts, (size_t)n_inst + 1));
    S_TRY(dalloc(&m->cursor, (size_t)n_inst + 1));
  }
  std::vector<char> hq((size_t)n_inst * isz);
  for (int i = 0; i < n_inst; ++i) mlp_qinst(k[i], a1[i], a2[i], (long)t_off[i], (long)t_off[i + 1], &hq[i * isz]);
  S_TRY(hipMemcpyAsync(m->qinst, hq.data(), hq.size(), hipMemcpyHostToDevice, m->stream));
  if ((size_t)T * 6 > m->qall_cap) {
    if (m->qall) (void)hipFree(m->qall);
    m->qall = nullptr;
    S_TRY(dalloc(&m->qall, (size_t)T * 6));
    m->qall_cap = (size_t)T * 6;
  }
  S_TRY(mlp_make_queries(m->stream, m->qinst, n_inst, x, T, m->qall));
  const size_t esz = info.prec == QPGF_C128 ? 16 : 8;
  // network on chunks of max_batch rows (fused kernel, every member per tile);
  // ensemble outputs side by side in ybuf
  const long ystride = m->maxb * 2;
  for (int64_t b0 = 0; b0 < T; b0 += m->maxb) {
    const long n = (long)std::min<int64_t>(m->maxb, T - b0);
    S_TRY(mlp_infer(m->stream, m->wb.data(), m->p.data(), m->members, B_OFF, OFF_W4, OFF_B4, info.c, info.c_tilde,
                    m->qall + 6 * b0, n, m->ybuf, ystride));
    S_TRY(mlp_combine(m->stream, info.prec, m->qall + 6 * b0, n, m->ybuf, m->members, m->maxb * 2, info.c, info.eps,
                      tol, m->kappa, wood_tol, rmin, static_cast<char*>(out) + b0 * esz, fell_back + b0));
  }
  // fallback: per-instance compaction, the plain method on those targets, scatter back
  std::vector<uint32_t> cnt(n_inst + 1, 0);
  S_TRY(hipMemsetAsync(m->counts, 0, (n_inst + 1) * sizeof(uint32_t), m->stream));
  hipLaunchKernelGGL(k_count_fallback, dim3(gb(T)), dim3(256), 0, m->stream, fell_back, m->qinst, n_inst, isz,
                     mlp_qinst_t0_offset(), (long)T, m->counts, m->cursor, m->counts, m->fidx, 0);
  S_TRY(hipGetLastError());
  S_TRY(hipMemcpyAsync(cnt.data(), m->counts, n_inst * sizeof(uint32_t), hipMemcpyDeviceToHost, m->stream));
  S_TRY(hipStreamSynchronize(m->stream));
  std::vector<uint32_t> offs(n_inst + 1, 0);
  for (int i = 0; i < n_inst; ++i) offs[i + 1] = offs[i] + cnt[i];
  const long nf = offs[n_inst];
  if (n_fallback) *n_fallback = nf;
  if (nf == 0) return QPGF_OK;
  if ((size_t)nf > m->fidx_cap) {
    if (m->fidx) (void)hipFree(m->fidx);
    m->fidx = nullptr;
    S_TRY(dalloc(&m->fidx, (size_t)nf));
    m->fidx_cap = (size_t)nf;
  }
  uint32_t* doffs = m->counts;   // reuse: offsets
  S_TRY(hipMemcpyAsync(doffs, offs.data(), (n_inst + 1) * sizeof(uint32_t), hipMemcpyHostToDevice, m->stream));
  S_TRY(hipMemsetAsync(m->cursor, 0, (n_inst + 1) * sizeof(uint32_t), m->stream));
  hipLaunchKernelGGL(k_count_fallback, dim3(gb(T)), dim3(256), 0, m->stream, fell_back, m->qinst, n_inst, isz,
                     mlp_qinst_t0_offset(), (long)T, m->counts, m->cursor, doffs, m->fidx, 1);
  S_TRY(hipGetLastError());
  size_t maxc = 0;
  for (int i = 0; i < n_inst; ++i) maxc = std::max(maxc, (size_t)cnt[i]);
  if (maxc > m->fx_cap) {
    if (m->fx) (void)hipFree(m->fx);
    if (m->fout) (void)hipFree(m->fout);
    m->fx = nullptr;
    m->fout = nullptr;
    S_TRY(dalloc(&m->fx, maxc * 3));
    S_TRY(hipMalloc(&m->fout, maxc * 16));
    m->fx_cap = maxc;
  }
  S_TRY(qpgf_plan_set_stream(plan, m->stream) == QPGF_OK ? hipSuccess : hipErrorInvalidValue);
  for (int i = 0; i < n_inst; ++i) {
    if (!cnt[i]) continue;
    hipLaunchKernelGGL(k_pick, dim3(gb(cnt[i])), dim3(256), 0, m->stream, x, m->fidx + offs[i], (long)cnt[i], m->fx);
    S_TRY(hipGetLastError());
    qpgf_status st = qpgf_gd3d(plan, k[i], a1[i], a2[i], m->fx, cnt[i], m->fout, nullptr);
    if (st != QPGF_OK) return sfail(st, std::string("fallback instance ") + std::to_string(i) + ": " + qpgf_last_error());
    hipLaunchKernelGGL(k_put, dim3(gb(cnt[i])), dim3(256), 0, m->stream, static_cast<const char*>(m->fout),
                       m->fidx + offs[i], (long)cnt[i], esz, static_cast<char*>(out));
    S_TRY(hipGetLastError());
  }
  return QPGF_OK;
}


// ---------------------------------------------------------------------------
// Training data, training loop, calibration of the error estimate, checkpoints
// ---------------------------------------------------------------------------
namespace {

qpgf_status fallback_plan(qpgf_mlp* m, qpgf_plan* plan, qpgf_plan_info& info) {
  if (qpgf_plan_get_info(plan, &info) != QPGF_OK || info.kind != QPGF_KIND_GD3D)
    return sfail(QPGF_E_ARG, "the plan must be of kind GD3D");
  if (info.c != kC || info.c_tilde != kCt)
    return sfail(QPGF_E_ARG, "the plan must use the surrogate's c = 0.6 and c_tilde = 1");
  if (qpgf_plan_set_stream(plan, m->stream) != QPGF_OK) return sfail(QPGF_E_ARG, "plan stream");
  return QPGF_OK;
}

qpgf_status check_instances(int n_inst, const double* k, const double* a1, const double* a2, const int64_t* t_off) {
  if (n_inst <= 0 || !k || !a1 || !a2 || !t_off) return sfail(QPGF_E_ARG, "bad instance arguments");
  if (t_off[0] != 0) return sfail(QPGF_E_ARG, "t_off[0] must be 0");
  for (int i = 0; i < n_inst; ++i)
    if (t_off[i + 1] < t_off[i]) return sfail(QPGF_E_ARG, "t_off must be non-decreasing");
  if (t_off[n_inst] > (int64_t)0x7fffffff) return sfail(QPGF_E_SIZE, "at most 2^31 - 1 targets");
  return QPGF_OK;
}

// prepare instance i and write the plain method's smooth part at its targets into L
qpgf_status smooth_of(qpgf_plan* plan, int i, double k, double a1, double a2, const double* x, int64_t n, void* L) {
  qpgf_status st = qpgf_prepare(plan, k, a1, a2);
  if (st == QPGF_OK && n > 0) st = qpgf_evaluate_smooth(plan, x, n, L);
  if (st != QPGF_OK)
    return sfail(st, std::string("instance ") + std::to_string(i) + ": " + qpgf_last_error());
  return QPGF_OK;
}

struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

constexpr char kCkptMagic[8] = {'Q', 'P', 'G', 'F', 'M', 'L', 'P', '1'};

}  // namespace

extern "C" {

qpgf_status qpgf_mlp_set_calibration(qpgf_mlp* m, double kappa) {
  s_err.clear();
  if (!m) return sfail(QPGF_E_ARG, "model is NULL");
  if (!(kappa > 0.0)) return sfail(QPGF_E_ARG, "kappa must be positive (+inf: accept nothing)");
  m->kappa = kappa;
  return QPGF_OK;
}

qpgf_status qpgf_mlp_get_calibration(const qpgf_mlp* m, double* kappa) {
  s_err.clear();
  if (!m || !kappa) return sfail(QPGF_E_ARG, "model and kappa must be non-NULL");
  *kappa = m->kappa;
  return QPGF_OK;
}

qpgf_status qpgf_surrogate_make_data(qpgf_mlp* m, qpgf_plan* plan, int n_inst, const double* k, const double* a1,
                                     const double* a2, const int64_t* t_off, const double* x, double* q, float* y) {
  s_err.clear();
  if (!m || !plan) return sfail(QPGF_E_ARG, "model and plan must be non-NULL");
  qpgf_status st = check_instances(n_inst, k, a1, a2, t_off);
  if (st != QPGF_OK) return st;
  qpgf_plan_info info;
  st = fallback_plan(m, plan, info);
  if (st != QPGF_OK) return st;
  const int64_t T = t_off[n_inst];
  if (T == 0) return QPGF_OK;
  if (!x || !q || !y) return sfail(QPGF_E_ARG, "x, q and y must be non-NULL");
  int64_t maxn = 0;
  for (int i = 0; i < n_inst; ++i) maxn = std::max(maxn, t_off[i + 1] - t_off[i]);
  DevBuf L;
  S_TRY(hipMalloc(&L.p, (size_t)maxn * 16));
  for (int i = 0; i < n_inst; ++i) {
    const int64_t t0 = t_off[i], n = t_off[i + 1] - t0;
    st = smooth_of(plan, i, k[i], a1[i], a2[i], x + 3 * t0, n, L.p);
    if (st != QPGF_OK) return st;
    if (n) S_TRY(mlp_make_rows(m->stream, info.prec, x + 3 * t0, (long)n, k[i], a1[i], a2[i], L.p, q + 6 * t0,
                               y + 2 * t0));
  }
  S_TRY(hipStreamSynchronize(m->stream));   // L is freed on return
  return QPGF_OK;
}

qpgf_status qpgf_surrogate_train(qpgf_mlp* m, const double* q, const float* y, int64_t N, const qpgf_train_cfg* cfg,
                                 float* loss) {
  s_err.clear();
  if (!m || !cfg) return sfail(QPGF_E_ARG, "model and cfg must be non-NULL");
  const int64_t B = cfg->batch;
  if (B < 64 || B % 64 || B > m->maxb) return sfail(QPGF_E_ARG, "batch must be a multiple of 64 <= max_batch");
  if (N < B || N > (int64_t)0xffffffff) return sfail(QPGF_E_ARG, "need batch <= N < 2^32 rows");
  if (!q || !y) return sfail(QPGF_E_ARG, "q and y must be non-NULL");
  if (cfg->steps < 0) return sfail(QPGF_E_ARG, "steps < 0");
  if (!(cfg->lr_max > 0.f) || !(cfg->lr_min >= 0.f) || cfg->lr_min > cfg->lr_max)
    return sfail(QPGF_E_ARG, "need 0 <= lr_min <= lr_max, lr_max > 0");
  if (cfg->member < -1 || cfg->member >= m->members) return sfail(QPGF_E_ARG, "member out of range");
  if ((size_t)N > m->perm_cap) {
    if (m->perm) (void)hipFree(m->perm);
    m->perm = nullptr;
    m->perm_cap = 0;
    S_TRY(dalloc(&m->perm, (size_t)N));
    m->perm_cap = (size_t)N;
  }
  std::vector<uint32_t> order((size_t)N);
  const int e0 = cfg->member < 0 ? 0 : cfg->member, e1 = cfg->member < 0 ? m->members : cfg->member + 1;
  for (int e = e0; e < e1; ++e) {
    uint64_t s = cfg->seed * 0x9E3779B97F4A7C15ull + 1000003ull * (uint64_t)e + 12345ull;
    for (int64_t i = 0; i < N; ++i) order[i] = (uint32_t)i;
    int64_t pos = N;
    for (int64_t t = 0; t < cfg->steps; ++t) {
      if (pos + B > N) {
        // a fresh data order each epoch (Fisher-Yates); the previous upload must be complete
        S_TRY(hipStreamSynchronize(m->stream));
        for (int64_t i = N - 1; i > 0; --i) std::swap(order[i], order[splitmix(s) % (uint64_t)(i + 1)]);
        S_TRY(hipMemcpyAsync(m->perm, order.data(), (size_t)N * sizeof(uint32_t), hipMemcpyHostToDevice, m->stream));
        pos = 0;
      }
      S_TRY(mlp_gather_rows(m->stream, q, y, m->perm + pos, (long)B, m->q, m->ybuf));
      pos += B;
      const double lr = cfg->lr_min + 0.5 * (cfg->lr_max - cfg->lr_min) * (1.0 + cos(M_PI * (double)t / cfg->steps));
      qpgf_status st = qpgf_mlp_train_step(m, e, m->q, m->ybuf, B, (float)lr, loss ? loss + e : nullptr);
      if (st != QPGF_OK) return st;
    }
  }
  S_TRY(hipStreamSynchronize(m->stream));   // the host data order is freed on return
  return QPGF_OK;
}

qpgf_status qpgf_surrogate_calibrate(qpgf_mlp* m, qpgf_plan* plan, int n_inst, const double* k, const double* a1,
                                     const double* a2, const int64_t* t_off, const double* x, double quantile,
                                     double safety, double* kappa) {
  s_err.clear();
  if (!m || !plan) return sfail(QPGF_E_ARG, "model and plan must be non-NULL");
  qpgf_status st = check_instances(n_inst, k, a1, a2, t_off);
  if (st != QPGF_OK) return st;
  if (!(quantile > 0.0 && quantile <= 1.0)) return sfail(QPGF_E_ARG, "quantile must be in (0, 1]");
  if (!(safety >= 1.0) || std::isinf(safety)) return sfail(QPGF_E_ARG, "safety must be finite and >= 1");
  if (m->members < 2) return sfail(QPGF_E_ARG, "the error estimate needs at least two members");
  qpgf_plan_info info;
  st = fallback_plan(m, plan, info);
  if (st != QPGF_OK) return st;
  const int64_t T = t_off[n_inst];
  if (T == 0 || !x) return sfail(QPGF_E_ARG, "no calibration targets");
  const size_t esz = info.prec == QPGF_C128 ? 16 : 8;
  DevBuf L, R, Q;
  S_TRY(hipMalloc(&L.p, (size_t)T * esz));
  S_TRY(hipMalloc(&R.p, (size_t)T * sizeof(double)));
  S_TRY(hipMalloc(&Q.p, (size_t)m->maxb * 6 * sizeof(double)));
  for (int i = 0; i < n_inst; ++i) {
    const int64_t t0 = t_off[i], n = t_off[i + 1] - t0;
    st = smooth_of(plan, i, k[i], a1[i], a2[i], x + 3 * t0, n, static_cast<char*>(L.p) + t0 * esz);
    if (st != QPGF_OK) return st;
  }
  // queries chunk by chunk (rows of one instance share (k, alpha)), network, ratio
  double* q = static_cast<double*>(Q.p);
  const long ystride = m->maxb * 2;
  for (int i = 0; i < n_inst; ++i) {
    for (int64_t b0 = t_off[i]; b0 < t_off[i + 1]; b0 += m->maxb) {
      const long n = (long)std::min<int64_t>(m->maxb, t_off[i + 1] - b0);
      S_TRY(mlp_make_rows(m->stream, info.prec, x + 3 * b0, n, k[i], a1[i], a2[i],
                          static_cast<char*>(L.p) + b0 * esz, q, m->out));
      S_TRY(mlp_infer(m->stream, m->wb.data(), m->p.data(), m->members, B_OFF, OFF_W4, OFF_B4, kC, kCt, q, n,
                      m->ybuf, ystride));
      S_TRY(mlp_calib_ratio(m->stream, info.prec, n, m->ybuf, m->members, ystride,
                            static_cast<char*>(L.p) + b0 * esz, static_cast<double*>(R.p) + b0));
    }
  }
  std::vector<double> r((size_t)T);
  S_TRY(hipMemcpyAsync(r.data(), R.p, (size_t)T * sizeof(double), hipMemcpyDeviceToHost, m->stream));
  S_TRY(hipStreamSynchronize(m->stream));
  // far targets (NaN) carry no estimate; +inf stays and keeps the model from accepting anything
  r.erase(std::remove_if(r.begin(), r.end(), [](double v) { return v != v; }), r.end());
  if (r.empty()) return sfail(QPGF_E_ARG, "no near-region calibration targets (|x3| <= 0.6)");
  const size_t j = std::min(r.size() - 1, (size_t)std::ceil(quantile * (double)r.size()) - 1);
  std::nth_element(r.begin(), r.begin() + (long)j, r.end());
  const double kap = safety * r[j];
  m->kappa = kap > 0.0 ? kap : HUGE_VAL;
  if (kappa) *kappa = m->kappa;
  return QPGF_OK;
}

qpgf_status qpgf_mlp_save(qpgf_mlp* m, const char* path) {
  s_err.clear();
  if (!m || !path) return sfail(QPGF_E_ARG, "model and path must be non-NULL");
  std::vector<float> buf((size_t)NPARAM * 3);
  S_TRY(hipStreamSynchronize(m->stream));
  FILE* f = fopen(path, "wb");
  if (!f) return sfail(QPGF_E_IO, std::string("cannot open ") + path + " for writing");
  const int32_t members = m->members;
  const int64_t np = NPARAM;
  bool ok = fwrite(kCkptMagic, 1, 8, f) == 8 && fwrite(&members, sizeof members, 1, f) == 1 &&
            fwrite(&np, sizeof np, 1, f) == 1 && fwrite(&m->kappa, sizeof m->kappa, 1, f) == 1;
  for (int e = 0; e < m->members && ok; ++e) {
    const int64_t step = m->step[e];
    hipError_t r = hipMemcpy(buf.data(), m->p[e], NPARAM * sizeof(float), hipMemcpyDeviceToHost);
    if (r == hipSuccess) r = hipMemcpy(buf.data() + NPARAM, m->m1[e], NPARAM * sizeof(float), hipMemcpyDeviceToHost);
    if (r == hipSuccess)
      r = hipMemcpy(buf.data() + 2 * NPARAM, m->m2[e], NPARAM * sizeof(float), hipMemcpyDeviceToHost);
    if (r != hipSuccess) {
      fclose(f);
      return sfail(QPGF_E_HIP, std::string("checkpoint copy: ") + hipGetErrorString(r));
    }
    ok = fwrite(&step, sizeof step, 1, f) == 1 && fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  }
  ok = (fclose(f) == 0) && ok;
  if (!ok) return sfail(QPGF_E_IO, std::string("write to ") + path + " failed");
  return QPGF_OK;
}

qpgf_status qpgf_mlp_load(qpgf_mlp* m, const char* path) {
  s_err.clear();
  if (!m || !path) return sfail(QPGF_E_ARG, "model and path must be non-NULL");
  FILE* f = fopen(path, "rb");
  if (!f) return sfail(QPGF_E_IO, std::string("cannot open ") + path);
  char magic[8];
  int32_t members = 0;
  int64_t np = 0;
  double kap = 0.0;
  bool ok = fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kCkptMagic, 8) == 0 &&
            fread(&members, sizeof members, 1, f) == 1 && fread(&np, sizeof np, 1, f) == 1 &&
            fread(&kap, sizeof kap, 1, f) == 1;
  if (!ok || members != m->members || np != NPARAM || !(kap > 0.0)) {
    fclose(f);
    return sfail(QPGF_E_IO, std::string(path) + " is not a checkpoint of a " + std::to_string(m->members) +
                                "-member model of this architecture");
  }
  std::vector<float> buf((size_t)NPARAM * 3 * members);
  std::vector<int64_t> steps(members);
  for (int e = 0; e < members && ok; ++e)
    ok = fread(&steps[e], sizeof(int64_t), 1, f) == 1 && steps[e] >= 0 &&
         fread(buf.data() + (size_t)e * 3 * NPARAM, sizeof(float), (size_t)NPARAM * 3, f) == (size_t)NPARAM * 3;
  ok = ok && fgetc(f) == EOF;
  fclose(f);
  if (!ok) return sfail(QPGF_E_IO, std::string(path) + " is truncated or corrupt");
  // the model changes only once the whole file has been read
  S_TRY(hipStreamSynchronize(m->stream));
  for (int e = 0; e < members; ++e) {
    const float* b = buf.data() + (size_t)e * 3 * NPARAM;
    S_TRY(hipMemcpy(m->p[e], b, NPARAM * sizeof(float), hipMemcpyHostToDevice));
    S_TRY(hipMemcpy(m->m1[e], b + NPARAM, NPARAM * sizeof(float), hipMemcpyHostToDevice));
    S_TRY(hipMemcpy(m->m2[e], b + 2 * NPARAM, NPARAM * sizeof(float), hipMemcpyHostToDevice));
    m->step[e] = steps[e];
    S_TRY(refresh(m, e));
  }
  m->kappa = kap;
  S_TRY(hipStreamSynchronize(m->stream));
  return QPGF_OK;
}

}  // extern "C"
