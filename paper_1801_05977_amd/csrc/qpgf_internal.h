// Internal declarations of libqpgf: plan layout, device helpers, kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <string>
#include <vector>

#include "../../include/qpgf.h"

namespace qpgf {

// ---------------------------------------------------------------------------
// complex helpers (FP64 work is done in double2; bulk storage in T2)
// ---------------------------------------------------------------------------
// Maxwell near fields: L_d and the second-derivative fields of Algorithm 4.1, pq = 11 22 33 12 13 23
// (kMxF); with params.maxwell_trace the 33 field is dropped and GG_33 follows from the trace
// tr GG = 3 G_d + k^-2 Laplacian G_d = 2 G_d off the lattice (kMxT).  The far slab of the Maxwell
// kind holds the six tensor entries of the series directly (kMxO).
constexpr int kMxF = 7;
constexpr int kMxT = 6;
constexpr int kMxO = 6;
// Far branch: the far slab is interpolated with the P-point Lagrange rule per axis (nodes
// base - (P/2 - 1) .. base + P/2; its first slice lies P/2 - 1 spacings below c): P = 8 in 2D and
// for complex128 in 3D, P = 4 for complex64 in 3D (on a finer slab).
template <typename T> constexpr int far_points() { return sizeof(T) == 4 ? 4 : 8; }

template <typename T> struct C2;
template <> struct C2<double> { using type = double2; };
template <> struct C2<float> { using type = float2; };
template <typename T> using cplx = typename C2<T>::type;

__host__ __device__ inline double2 mk(double r, double i) { return make_double2(r, i); }
__host__ __device__ inline double2 cadd(double2 a, double2 b) { return mk(a.x + b.x, a.y + b.y); }
__host__ __device__ inline double2 csub(double2 a, double2 b) { return mk(a.x - b.x, a.y - b.y); }
__host__ __device__ inline double2 cmul(double2 a, double2 b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__host__ __device__ inline double2 cscale(double2 a, double s) { return mk(a.x * s, a.y * s); }
// Smith's algorithm: a / b without overflow for large |b|.
__host__ __device__ inline double2 cdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return mk((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  double r = b.x / b.y, d = b.x * r + b.y;
  return mk((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
// e^{i z} for complex z.
__device__ inline double2 cexpi(double2 z) {
  double s, c;
  sincos(z.x, &s, &c);
  double m = exp(-z.y);
  return mk(m * c, m * s);
}
// beta = sqrt(k^2 - rho^2) on the branch Im beta >= 0 (Section 1), evaluated as
// sqrt((k - rho)(k + rho)) so it does not cancel near a Wood anomaly.
__host__ __device__ inline double2 beta_of(double k, double rho) {
  double d = (k - rho) * (k + rho);
  return d >= 0.0 ? mk(sqrt(d), 0.0) : mk(0.0, sqrt(-d));
}

// The far slab's evanescent terms (c/q) e^{-qz} with q z > kFarNegligibleQz are taken as zero.  The
// modes lie one per unit area of the (xi1, xi2) plane, so the dropped terms sum to about
// 2 pi c e^{-50} / z (about 1e-21 c / z), against the propagating terms' c/p >= c/k: far below the
// FP64 rounding of the slab's values.  The Maxwell entries carry at most 1 + |xi|^2/k^2 more, so
// theirs sum to about 3e-18 c/(k^2 z^3).  The test takes |xi|^2 = r2, before any square root
// (q^2 = r2 - k^2).  A column j1 past it with r2 = (alpha1 + j1)^2 has every term (any j2) past it
// too, up to the rounding of terms at the cut itself.
constexpr double kFarNegligibleQz = 50.0;
__host__ __device__ inline bool far_negligible(double r2, double k, double z) {
  return (r2 - k * k) * (z * z) > kFarNegligibleQz * kFarNegligibleQz;
}
// Whether the far slab's column j1 (xi = alpha1 + j1), or Maxwell row j2 (xi = alpha2 + j2), at
// slice s holds only terms past the cut: far_negligible with |xi|^2 = xi^2 at z = z0 + s hf.  It
// decides which values the first transform writes and the second reads, so it is evaluated without
// contraction: every kernel that calls it takes the same decision, bit for bit.
__host__ __device__ inline bool far_band_empty(double xi, double k, double z0, double hf, long s) {
#pragma clang fp contract(off)
  const double z = z0 + (double)s * hf;
  return (xi * xi - k * k) * (z * z) > kFarNegligibleQz * kFarNegligibleQz;
}

// ---------------------------------------------------------------------------
// C^8 cut-off transition S(u) = I_u(9,9) (Bernstein form), S', S''
// ---------------------------------------------------------------------------
__host__ __device__ inline double smooth_S(double u) {
  if (u <= 0.0) return 0.0;
  if (u >= 1.0) return 1.0;
  // sum_{j=9}^{17} C(17,j) u^j (1-u)^{17-j}
  const double binom[9] = {24310.0, 19448.0, 12376.0, 6188.0, 2380.0, 680.0, 136.0, 17.0, 1.0};
  double v = 1.0 - u, s = 0.0;
  double uj = 1.0;
  for (int j = 0; j < 9; ++j) uj *= u;  // u^9
  double vp[9];
  vp[0] = 1.0;
  for (int j = 1; j < 9; ++j) vp[j] = vp[j - 1] * v;  // v^0..v^8
  for (int j = 9; j <= 17; ++j) {
    s += binom[j - 9] * uj * vp[17 - j];
    uj *= u;
  }
  return s;
}
__host__ __device__ inline double smooth_S1(double u) {
  if (u <= 0.0 || u >= 1.0) return 0.0;
  double w = u * (1.0 - u), w2 = w * w, w4 = w2 * w2;
  return 218790.0 * w4 * w4;
}
__host__ __device__ inline double smooth_S2(double u) {
  if (u <= 0.0 || u >= 1.0) return 0.0;
  double w = u * (1.0 - u), w2 = w * w, w4 = w2 * w2;
  return 218790.0 * 8.0 * w4 * w2 * w * (1.0 - 2.0 * u);
}
// Y_eps(r) = 1 - S((r - eps)/eps) and its radial derivatives.
__host__ __device__ inline double cut_Y(double r, double eps) { return 1.0 - smooth_S((r - eps) / eps); }
__host__ __device__ inline double cut_Y1(double r, double eps) { return -smooth_S1((r - eps) / eps) / eps; }
__host__ __device__ inline double cut_Y2(double r, double eps) { return -smooth_S2((r - eps) / eps) / (eps * eps); }

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
// One batched inverse-FFT segment (see k_fft_multi): `nbatch` transforms of
// length n starting at element `off`; transform b starts at
// (b / b_in) * s_out + (b % b_in) * s_in, elements `es` apart; `tile` transforms
// per block; the segment's first block is blk0.
struct FftSeg {
  long off;
  int n;
  long es, nbatch, b_in, s_in, s_out;
  int tile;
  long blk0;
};
constexpr int kMaxLog2 = 12;   // m <= 4096
// Twiddle table length: every transform length n = 2^a r (a <= 12, r in {1, 3, 5, 7}) divides it.
constexpr int kTwiddles = (1 << kMaxLog2) * 3 * 5 * 7;

// Per-call target scratch of the gathers.
struct TargetScratch {
  bool ext = false;                    // not owned by the plan: never grown or freed
  int64_t bin_cap = 0;                 // targets the per-target arrays hold
  int bin_keycap = 0;                  // keys hist / offs hold
  int bin_cntkeys = 0;                 // keys the per-(block, key) counts hold (LDS-histogram binning)
  uint2* bin_keyrank = nullptr;
  void* bin_rec = nullptr;             // targets in tile order (32-byte records)
  uint32_t* bin_hist = nullptr;
  uint32_t* bin_offs = nullptr;
  uint32_t* bin_cnt = nullptr;         // per-(block, key) counts / bases
  uint32_t* bin_ovf = nullptr;         // sorted positions handed to the overflow kernel
  uint32_t* bin_novf = nullptr;        // their count
  unsigned long long* ring_mask = nullptr;  // 2D kinds, ring_interp: one bit per target, set for the
  int64_t ring_words = 0;                   // targets of the cut-off ring (ring_words 64-bit words)
};

struct Plan {
  qpgf_params p;
  int dim = 2, nf = 1;         // nf: number of near fields (kMxF or kMxT for Maxwell)
  int M1 = 0, M2 = 0, M3 = 1;  // 2D: M3 = 1, M2 = transverse
  int Mt = 0;                  // transverse size (M2 in 2D, M3 in 3D)
  int S = 0;                   // far-slab slices
  int Mf1 = 0, Mf2 = 1;        // far-slab modes per periodic axis (Mf2 = 1 in 2D)
  int nfo = 1;                 // far-slab fields (kMxO for Maxwell, else nf)
  int fp = 8;                  // far-slab interpolation points per axis
  double hf = 0.0, fz0 = 0.0;  // far-slab slice spacing and first slice c - (fp/2 - 1) hf
  size_t far_cap = 0;          // bytes allocated for the far slab (grown when an instance needs more)
  size_t ncell = 0;            // points per near field
  size_t nfar = 0;             // points per far field
  size_t esize = 16;           // bytes per complex element
  hipStream_t stream = nullptr;

  // device buffers
  void* grid = nullptr;        // nf * ncell complex
  void* far = nullptr;         // nf * nfar complex
  double* xq = nullptr;        // X' quadrature nodes on [c, (c+c~)/2]
  double* wxq = nullptr;       // weights * X'(node)
  double* wXq = nullptr;       // weights * X(node) (special coefficients)
  double2* cs = nullptr;       // [Nt+1][Q]: (cos, sin)(j pi/c~ * xq)
  double* rq = nullptr;        // radial quadrature nodes on [eps, 2 eps]
  double* wrq = nullptr;       // weights
  double* y1q = nullptr;       // Y'(rq)
  double* y2q = nullptr;       // Y''(rq)
  double2* tw = nullptr;       // twiddles e^{2 pi i j / ntw}, double
  float2* twf = nullptr;       // same, float
  int ntw = 0;
  double2* F1 = nullptr;       // 2D singular tables (FFT order [j2'][j1'])
  double2* F2 = nullptr;
  size_t gridI_bytes = 0;      // its size (0: none)
  void* farI = nullptr;        // 2D plans with gridI: the far slab in the same layout (node quads or
  size_t farI_cap = 0;         // fields interleaved per node), grown with the slab
  // caller-owned workspace (qpgf_plan_set_workspace): grid, gridI, far and the target scratch
  // live in it; instances up to ws_kmax and calls of up to ws_T targets fit
  char* ws = nullptr;
  size_t ws_bytes = 0;
  double ws_kmax = 0.0;
  int64_t ws_T = 0;
  void* gridI = nullptr;       // 2D derivative kinds: the near fields interleaved, [i2][i1][field];
                               // complex64 G: node quads [i2][i1][a] = grid[i2][i1 + a]
  double* E2 = nullptr;        // 2D G with sing_order >= 2: [4][j2'][j1'] real tables of the removed
                               // degree-2 and degree-3 terms (e_tt, e_rr, e_ttt, e_trr)
  double* D2 = nullptr;        // 2D derivative tables: gradient [8][j2'][j1'] (a1 P1 Q1 R1 a2 P2 Q2 R2),
                               // second-derivative differences [6][j2'][j1'] (u11 v11 u12 v12 u22 v22)
  double2* htab = nullptr;     // 3D: H(rho) on rho = (m - 4) dh
  int Qr = 0;                  // nodes of the radial rule rq, wrq, y1q, y2q
  int hn = 0;
  double hd = 0.05;
  double last_k = 0, last_a1 = 0, last_a2 = 0;
  double last_k2 = 0;          // second wavenumber (differences of second derivatives)
  bool spec = false;           // the prepared instance has a special coefficient (fills take that path)
  bool prepared = false;

  // target binning scratch (3D) and ring mask (2D ring_interp): grown on demand while the plan
  // owns it (scratch_ext false); otherwise memory the plan does not own (a caller's workspace, or
  // the library's fixed scratch during one call), whose capacities are never exceeded
  int64_t bin_min_targets = 1 << 16;   // bin when T >= this; < 0 never
  TargetScratch ts;
  // tile configuration of the last binning (launch_bin3d), used by launch_gather_binned
  int bt[24] = {};                     // the tile configuration (near and far tiles, key counts)
  int64_t bt_T = -1;
  const double* bt_x = nullptr;
  // second stream for the binning while the grids are prepared, and its events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  // FFT tiles chosen by the autotuner: key (n << 2) | rows | c64 << 1
  std::map<int, int> fft_tiles;

  // batched 2D: instance grids, descriptors, the captured graph
  void* b_grid = nullptr;
  void* b_far = nullptr;
  size_t b_grid_cap = 0, b_far_cap = 0;   // bytes
  void* b_desc = nullptr;                  // device descriptors
  void* b_host = nullptr;                  // pinned staging for them
  size_t b_desc_cap = 0;
  hipEvent_t b_upload_done = nullptr;
  hipStream_t b_capture = nullptr;
  hipGraph_t b_graph = nullptr;
  hipGraphExec_t b_exec = nullptr;
  std::vector<int64_t> b_sig;              // n, m1[], t_off[], pointers of the captured graph

  // per-kernel timing (qpgf_plan_enable_timing)
  struct Pending { int id; hipEvent_t a, b; };
  bool timing = false;
  int device = 0;              // the GPU the plan's arrays live on (current at creation)
  std::vector<Pending> pending;
  double t_ms[QPGF_T_COUNT] = {};
  int64_t t_n[QPGF_T_COUNT] = {};
};

// Brackets one launch with events on the plan's stream when timing is on.
struct KernelTimer {
  Plan& P;
  int id;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  // events on stream st (default: the plan's stream)
  KernelTimer(Plan& p, int i, hipStream_t st = nullptr) : P(p), id(i), s(st ? st : p.stream) {
    if (P.timing && hipEventCreate(&a) == hipSuccess && hipEventCreate(&b) == hipSuccess)
      (void)hipEventRecord(a, s);
    else
      a = b = nullptr;
  }
  ~KernelTimer() {
    if (a && b) {
      (void)hipEventRecord(b, s);
      P.pending.push_back({id, a, b});
    }
  }
};

// Far-slab geometry for an instance whose largest wavenumber is kmax and whose x1 (2D) or x1, x2
// (3D) near sizes are M1 (and P.M2): modes per periodic axis and slice spacing (api.hip).
struct FarGeom {
  int Mf1, Mf2, S;
  int P;          // interpolation points per axis
  double hf;
};
FarGeom far_geometry(const Plan& P, double kmax, int M1);

// kernel launchers (fill.hip, fft.hip, gather.hip)
hipError_t launch_interleave2d(Plan& P);
hipError_t launch_sing2d_ho(Plan& P, int Qg, const double* rg, const double* wyg);
hipError_t launch_sing2d_hess(Plan& P, int Qg, const double* rg, const double* wyg);
hipError_t launch_sing2d_grad(Plan& P, int Qg, const double* rg, const double* wyg);
hipError_t launch_sing2d(Plan& P, double f1_zero);
hipError_t launch_htable(Plan& P, double k);
hipError_t launch_fill(Plan& P, double k, double a1, double a2, bool fuse_transverse);
bool fill_fuses_transverse(const Plan& P);
bool far_rows_in_fill(const Plan& P);
bool far7_ok(const Plan& P);
hipError_t launch_far(Plan& P, double k, double a1, double a2);
// x1 rows of the 3D G_d far slab after its x2 pass, reading only the columns that hold terms
hipError_t launch_fft_far_rows(Plan& P, double k, double a1);
// x2 columns of the Maxwell far slab after its x1 pass, reading only the rows that hold terms
hipError_t launch_fft_far_cols(Plan& P, double k, double a2);
hipError_t launch_fft(Plan& P, void* data, int n, long elem_stride, long nbatch, long b_in, long s_in,
                      long s_out);
int fft_tile(const Plan& P, int n, bool rows, long nbatch);
// batched 2D (one launch per stage for many instances)
void fill_inst_2d(const Plan& P, double k, double a, int M1, const FarGeom& fg, long off, long foff, long blk0,
                  void* dst);
size_t fill_inst_size();
hipError_t launch_fill2d_multi(Plan& P, const void* dinst, int n_inst, long nblocks, void* base, bool spec);
hipError_t launch_far2d_multi(Plan& P, const void* dinst, int n_inst, long nblocks, void* base);
void gather_inst_2d(const Plan& P, double k, double a, int M1, const FarGeom& fg, long off, long foff, long t0,
                    long t1, long blk0, void* dst);
size_t gather_inst_size();
hipError_t launch_gather2d_multi(Plan& P, const void* dinst, int n_inst, long nblocks, const void* grid,
                                 const void* far, const double* x, void* out, uint8_t* flags);
hipError_t launch_fft_multi(Plan& P, void* base, const FftSeg* dsegs, int nseg, long nblocks, long lds_elems);
hipError_t launch_gather(Plan& P, const double* x, int64_t T, void* out, uint8_t* flags);
hipError_t ensure_bin_scratch(Plan& P, int64_t T, int nkeys);
hipError_t ensure_ring_scratch(Plan& P, int64_t T);
// Upper bound of the binning keys of any 3D evaluate on far slabs up to (Mf1, Mf2, S) (0 for 2D).
int bin_keys_bound(const Plan& P, int Mf1, int Mf2, int S, int fp);
// Lay out target scratch for T targets and nkeys keys at base (256-byte aligned; NULL: only size
// it); returns the bytes used.  With base set, ts points into it (ext = true).
size_t carve_target_scratch(const Plan& P, char* base, int64_t T, int nkeys, TargetScratch& ts);
void free_target_scratch(TargetScratch& ts);
hipError_t launch_gather_smooth(Plan& P, const double* x, int64_t T, void* out);
// The 3D calculation step in two halves: binning of the targets by grid tile
// (needs only the targets and the plan's geometry, so it may run on another
// stream while the grids are prepared) and the tiled gather on the plan's stream.
bool gather_uses_bins(const Plan& P, int64_t T);
hipError_t launch_bin3d(Plan& P, const double* x, int64_t T, hipStream_t stream);
hipError_t launch_gather_binned(Plan& P, const double* x, int64_t T, void* out, uint8_t* flags);

}  // namespace qpgf
