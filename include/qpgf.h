/*
 * qpgf.h -- C ABI of libqpgf, the MI355X (gfx950) implementation of the
 * FFT-based evaluator of quasi-periodic Green's functions of Zhang & Zhang,
 * "An FFT-based algorithm for efficient computation of Green's functions for
 * the Helmholtz and Maxwell's equations in periodic domains".
 *
 * Functions evaluated (Section 1 of the paper):
 *   G(x; k, alpha)            2D, 2pi-periodic in x1, alpha-quasi-periodic, eq. (1.2)
 *   G_d(x; k, alpha1, alpha2) 3D, 2pi-periodic in x1 and x2, eq. (1.3)
 *   GG(x) = G_d I + k^-2 grad grad G_d, the Maxwell Green tensor, eq. (1.4)
 * for k > 0, real alpha, away from Wood anomalies (beta_n != 0, Section 1).
 *
 * Method (Algorithms 2.1, 3.1, 4.1): preparation fills the Fourier
 * coefficients L-hat = K-hat - F-hat of the periodised, desingularised
 * function (eqs. 2.1-2.5, 3.3, 3.5, Section 4) in FP64 and transforms them to
 * a uniform grid with inverse FFTs; evaluation reduces each target to the
 * period cell, interpolates the grid with the 4-point cubic Lagrange rule per
 * axis (16 / 64 points) and adds back the removed singular part exactly and the
 * quasi-periodic phase.  Targets with |x_t| > c (x_t = x2 in 2D, x3 in 3D) take
 * the far branch, where step 2b of the algorithms uses the eigenfunction series
 * itself: the series' terms are summed by inverse FFT on a far slab of slices
 * z_s = c - (P/2 - 1) h_f + s h_f, s = 0 .. S_f-1, with far_m modes per periodic
 * axis, and the slab is interpolated with the P-point Lagrange rule per axis: P = 8
 * (64 / 512 nodes), or P = 4 (64 nodes, on a finer slab) for complex64 in 3D.  No singular part exists there; with the automatic slab geometry (far_m,
 * far_h) the far branch agrees with the direct sum of the series to about 1e-11
 * (complex128) or 1e-7 (complex64) relative.
 *
 * Conventions for every entry point:
 *  - All bulk arrays (targets, outputs, flags) are DEVICE pointers owned by the
 *    caller.  The plan owns its grids, coefficient tables and scratch, which it
 *    allocates with hipMalloc at creation (grids) or on first use (target
 *    scratch, grown as needed).
 *  - Work is enqueued asynchronously on the plan's stream (default: the null
 *    stream); the return value reports launch-time validation and HIP launch
 *    errors only.  Calls on one plan must not overlap from several host threads.
 *  - Targets are float64, row-major [T][dim].  Outputs are interleaved complex
 *    (re, im) in the caller's target order: complex128 when the plan precision is
 *    QPGF_C128, complex64 when QPGF_C64.  Maxwell outputs are [T][6] complex in
 *    the order 11, 22, 33, 12, 13, 23.  The plan carries the seven fields of
 *    Algorithm 4.1 (L_d and L^{pq} for pq = 11, 22, 33, 12, 13, 23), unless
 *    params.maxwell_trace asks for the six-field variant.
 *  - Per-target flags (optional, may be NULL), uint8 [T]:
 *      bit 0  the target lies within params.lattice_rmin of a lattice point
 *             (output NaN); with lattice_rmin = 0 only an exact hit is flagged,
 *      bit 1  far branch (|x_t| > c),
 *      bit 2  |x_t| beyond the far slab, i.e. >= c + (S_f - P + 1) h_f (output NaN;
 *             the slab covers |x_t| <= params.far_zmax),
 *      bit 3  non-finite target coordinate (output NaN).
 *  - On error the call returns a nonzero qpgf_status and qpgf_last_error()
 *    describes it; nothing is launched.
 */
#ifndef QPGF_H
#define QPGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QPGF_OK = 0,
  QPGF_E_ARG = 1,          /* invalid argument (null pointer, bad size, wrong plan kind) */
  QPGF_E_WOOD = 2,         /* min_n |beta_n| < wood_tol: Wood anomaly (Section 1)        */
  QPGF_E_SPECIAL = 3,      /* kept for the ABI; no longer returned: the special
                              coefficients beta = -+j pi/c~ are evaluated (special_tol)  */
  QPGF_E_SIZE = 4,         /* unsupported grid size                                      */
  QPGF_E_HIP = 5,          /* a HIP runtime call failed                                  */
  QPGF_E_NOMEM = 6,        /* device allocation failed                                   */
  QPGF_E_UNSUPPORTED = 7,
  QPGF_E_IO = 8            /* a checkpoint file could not be opened, read or written, or
                              is not a checkpoint of this model                          */
} qpgf_status;

typedef enum { QPGF_C128 = 0, QPGF_C64 = 1 } qpgf_prec;

typedef enum {
  QPGF_KIND_G2D = 0,       /* Algorithm 2.1 */
  QPGF_KIND_GD3D = 1,      /* Algorithm 3.1 */
  QPGF_KIND_MAXWELL3D = 2, /* Algorithm 4.1 */
  QPGF_KIND_G2D_GRAD = 3,  /* first derivatives of the 2D G (Section 2.4.1) */
  QPGF_KIND_G2D_HESS_DIFF = 4  /* differences of second derivatives of the 2D G for two
                                  wavenumbers (Section 2.4.2) */
} qpgf_kind;

/* Method parameters.  Grid sizes follow Sections 2.1 / 3.1 with an independent
 * size per axis: m1 = 2 N1 modes in x1; 2D: m2 = 2 N2 transverse (x2) modes;
 * 3D: m2 = 2 N2 modes in x2 and m3 = 2 N3 transverse (x3) modes.  Each must be
 * a power of two in [16, 4096] (m3 unused in 2D), except m1 of the 2D kinds:
 * 2^a r with a >= 1 and r in {1, 3, 5, 7} (the transforms' radix-3, -5 and -7
 * passes follow the power-of-two ones), in [16, 4096]; with complex128 the axes
 * transformed as columns (2D: m2; 3D: m2, m3) at most 2048.  Grid spacing: pi/N1, pi/N2
 * (3D) and c_tilde/N_t in the transverse direction.
 * Defaults (qpgf_params_default): c = 0.6, c_tilde = 1 (the values of Section 6),
 * eps = 0.2, cut-offs: C^8 smoothstep I_u(9,9) transitions (Section 6 states C^8),
 * quad_q = 64, far_h = 0 and far_m = 0 (the far slab's geometry follows each instance's
 * wavenumber, see far_m), far_zmax = c_tilde, wood_tol = 1e-3, special_tol = 1e-2,
 * lattice_rmin = 0, maxwell_trace = 0.
 * special_tol: a coefficient whose propagating beta lies within special_tol of |J|
 * (J = j_t pi / c~; the special cases of Sections 2.1 / 3.1, where the integration
 * by parts behind eqs. 2.1 / 3.3 divides by beta -+ J and loses digits close to it)
 * is computed from the integral that defines it, (i/(2 beta)) [I0(beta - J) +
 * I0(beta + J)] A, I0(g) = int_0^{c~} e^{igx} X(x) dx (the paper's special-case
 * formula), and in 3D the singular part's coefficient, 0/0 at |xi| = k in eq. 3.5,
 * from the radial transform of e^{ikr} Y/(4 pi r).  No instance is refused for it. */
typedef struct {
  int kind;                /* qpgf_kind */
  int prec;                /* qpgf_prec: precision of grids, FFTs, gather and output */
  int m1, m2, m3;
  double c;                /* near/far threshold and start of the X cut-off transition */
  double c_tilde;          /* periodisation half-length in the transverse axis, c_tilde > c */
  double eps;              /* singular cut-off Y_eps: 1 on [0, eps], 0 beyond 2 eps; 2 eps <= c_tilde */
  int quad_q;              /* Gauss-Legendre nodes for the X'- and radial integrals, 16..256 */
  double far_h;            /* far-slab slice spacing h_f; 0: automatic, the largest 2^-j <= min(1/64, x/k),
                              x = 0.107 for complex128 and 0.11 for complex64 */
  double far_zmax;         /* largest |x_t| the far slab must cover */
  double wood_tol;
  double special_tol;
  double lattice_rmin;
  int sing_order;          /* QPGF_KIND_G2D: highest degree m of the Taylor factor of the removed log
                              singularity -(1/2pi) ln r J0(k r) e^{-i alpha x1} (Remark 5.3).  1 (default)
                              removes 1 - i alpha x1 (f1, f2 of Section 2.2, Algorithm 2.1 as printed); 2
                              adds -(alpha^2/2) x1^2 - (k^2/4) r^2; 3 adds i (alpha^3/6) x1^3 + i (alpha k^2/4)
                              x1 r^2.  The remainder is O(r^{m+1} ln r), so near a lattice point the error
                              falls like N^-(m+1) instead of N^-2.  Every other kind requires 1. */
  int ring_interp;         /* QPGF_KIND_G2D (single-instance calls), QPGF_KIND_G2D_GRAD, QPGF_KIND_G2D_HESS_DIFF:
                              1 interpolates K = L + f Y (f the removed singular part; for the derivative
                              kinds L_p + h_p, L_pq + h_pq)
                              instead of L for near targets with r_lo < r < r_hi, r_hi =
                              2 eps + 2 sqrt(2) h, r_lo = max(eps, eps/2 + 2 sqrt(2) h), h = max(h1, h2) (every
                              stencil node then stays eps/2 or more from the lattice point), and adds nothing
                              back there.  L carries the steep transition of
                              Y_eps times the logarithm across that ring, K does not (Remark 5.6 ties the
                              accuracy to the cut-offs' smoothness): the ring's error falls by two to three
                              orders of magnitude.  The gather marks those targets (one bit per target in a
                              plan-owned mask of T/8 bytes, grown on demand) and a second pass corrects them
                              in FP64 (both precisions).
                              0 (default): Algorithm 2.1 / Section 2.4 as printed.  Every
                              other kind, and qpgf_g2d_batched, require 0. */
  int far_m;               /* modes per periodic axis of the far slab (a power of two in [16, 4096],
                              complex128 x2 axis <= 2048); 0: automatic per prepared instance, the
                              largest of m1 rounded up to a power of two (3D x2: m2), a floor, and the
                              smallest power of two >= 2 pi k / x, x = 0.0977 for complex128 and 0.081
                              for complex64 (k: the instance's largest wavenumber).  The floor is 512
                              modes, 256 for complex64 in 2D.
                              The far slab holds the terms of the series with
                              |j| < far_m / 2; the 8-point rule interpolates a term of wavenumber q to
                              about (q h)^8 / 1000, h = 2 pi / far_m or h_f, which the automatic choice keeps
                              near 1e-11 (complex128) or 1e-7 (complex64) relative.  The slab is allocated
                              at plan creation for the smallest geometry and grown (synchronously) by
                              an instance that needs more. */
  int maxwell_trace;       /* QPGF_KIND_MAXWELL3D: 0 (default) carries the seven fields of Algorithm 4.1;
                              1 drops the 33 field and takes GG_33 = 2 G_d - GG_11 - GG_22 from the trace
                              (tr GG = 3 G_d + k^-2 Laplacian G_d = 2 G_d off the lattice: the Helmholtz
                              equation); one transform and one interpolated field fewer, a different
                              approximation of GG_33 near the plane.  Other kinds require 0. */
} qpgf_params;

typedef struct qpgf_plan qpgf_plan;

/* Plan description returned by qpgf_plan_get_info. */
typedef struct {
  int kind, prec, m1, m2, m3;
  int far_slices;          /* S_f */
  double far_h;
  double c, c_tilde, eps;
  int n_fields;            /* near fields: 1; 7 for Maxwell (L and L^{pq}, pq = 11 22 33 12 13 23),
                              6 with maxwell_trace (no 33); 2 for G2D_GRAD; 3 for G2D_HESS_DIFF */
  size_t grid_bytes;       /* bytes of one near-grid field */
  size_t far_grid_bytes;   /* bytes of one far-slab field */
  int far_m1, far_m2;      /* far-slab modes per periodic axis (far_m2 = 1 in 2D) */
  int far_fields;          /* far-slab fields: as n_fields, except Maxwell: 6, the tensor entries
                              GG_pq of the series (11 22 33 12 13 23; 13 and 23 for x3 > 0) */
  int far_points;          /* interpolation points per axis on the far slab: 8, or 4 for complex64
                              in 3D; slice s lies at |x_t| = c - (far_points/2 - 1) h_f + s h_f */
  int far_points_t;        /* points along x2 and x3 of the binned far gather for the last prepared
                              instance: 7 for the complex128 G_d where the slab's spacing h gives
                              k h <= 0.07 on both axes (the first 7 nodes of each 8-point row;
                              far tiles within 0.8 of a lattice point keep 8), else far_points */
} qpgf_plan_info;

/* Fill *p with the defaults above for the given kind, precision and sizes. */
void qpgf_params_default(qpgf_params* p, int kind, int prec, int m1, int m2, int m3);

/* Validate *p, allocate the plan's device buffers on the current HIP device and
 * compute its parameter-only tables (quadrature nodes, FFT twiddles, and in 2D
 * the k- and alpha-independent singular coefficients F-hat_1, F-hat_2 of
 * eqs. 2.4 / 2.5, which Remark 2.1 lets one precompute once; for
 * QPGF_KIND_G2D_GRAD and QPGF_KIND_G2D_HESS_DIFF instead the k- and
 * alpha-independent parts of the coefficients of the singular parts of Sections
 * 2.4.1 / 2.4.2).  Synchronous.
 * *out receives the plan; release it with qpgf_plan_destroy. */
qpgf_status qpgf_plan_create(const qpgf_params* p, qpgf_plan** out);

/* Free every device buffer of the plan (synchronises its stream first). */
void qpgf_plan_destroy(qpgf_plan* plan);

/* Set the HIP stream (hipStream_t passed as void*) all later work is enqueued on. */
qpgf_status qpgf_plan_set_stream(qpgf_plan* plan, void* hip_stream);

qpgf_status qpgf_plan_get_info(const qpgf_plan* plan, qpgf_plan_info* info);

/* Preparation step of Algorithm 2.1 / 3.1 / 4.1 for one instance: fill the
 * coefficients L-hat (and L-hat^{pq}) in FP64, inverse-FFT them to the near
 * grid, and build the far-slab grid.  a2 is ignored in 2D.  The grids stay in
 * the plan until the next prepare.  Returns QPGF_E_WOOD when the instance is
 * excluded (checked on the host before any launch). */
qpgf_status qpgf_prepare(qpgf_plan* plan, double k, double a1, double a2);

/* Calculation step (Algorithm 2.1 / 3.1 / 4.1 step 2) for T targets against the
 * last prepared instance.  x: device float64 [T][dim]; out: device complex
 * ([T], [T][6] for MAXWELL3D, [T][2] for G2D_GRAD, [T][3] for G2D_HESS_DIFF);
 * flags: device uint8 [T] or NULL.  T = 0 is a no-op. */
qpgf_status qpgf_evaluate(qpgf_plan* plan, const double* x, int64_t T, void* out, uint8_t* flags);
/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): qpgf_evaluate with the
 * same arguments, kernels and results, whose per-call target scratch (the
 * binning of 3D targets, the ring mask of 2D ring_interp) lives in a fixed
 * 64 MiB device array of the library instead of memory the plan allocates.
 * Each GPU the library runs on holds its own copy of that array until the
 * process ends (the first call on a device looks its address up).  The call
 * allocates nothing; the plan's grids must exist (a prepare before it, on a
 * plan that owns its arrays or has a workspace).  Every call on one GPU, from
 * any plan, shares that GPU's array: calls that overlap in time on one GPU
 * (other streams, other threads) race and must be serialised by the caller.
 * The scratch is cleared by the call's own kernels where it must start at
 * zero.  The plan's device must be current.  Errors: as qpgf_evaluate, and
 * QPGF_E_SIZE when the scratch of T targets does not fit (the message gives
 * the most that do for this plan: about 1e6 for a 256 x 256 x 64 GD3D plan). */
qpgf_status qpgf_evaluate_noalloc(qpgf_plan* plan, const double* x, int64_t T, void* out, uint8_t* flags);

/* prepare + evaluate: G (kind G2D), G_d (GD3D) and GG (MAXWELL3D) at T targets. */
qpgf_status qpgf_g2d(qpgf_plan* plan, double k, double alpha,
                     const double* x, int64_t T, void* out, uint8_t* flags);
qpgf_status qpgf_gd3d(qpgf_plan* plan, double k, double alpha1, double alpha2,
                      const double* x, int64_t T, void* out, uint8_t* flags);
qpgf_status qpgf_maxwell3d(qpgf_plan* plan, double k, double alpha1, double alpha2,
                           const double* x, int64_t T, void* out, uint8_t* flags);

/* prepare + evaluate of the gradient of the 2D G (Section 2.4.1), plan of kind
 * QPGF_KIND_G2D_GRAD.  K1 = e^{-i alpha x1} dG/dx1 and K2 = e^{-i alpha x1} dG/dx2
 * are periodic like K; the plan's two fields hold K_p - h_p (coefficients
 * i(alpha + j1) K-hat_j - H-hat_1j and i j2 (pi/c~) K-hat_j - H-hat_2j, the
 * Fourier coefficients H-hat of the singular parts h1, h2 from the plan's
 * tables), and the far slab the series (1.2) differentiated term by term.  At a
 * target the 16-point interpolant of each field plus h_p in FP64 (r < 2 eps),
 * times e^{i alpha x1}; beyond c the far slab, times sgn(x2) for x2.  h2 is
 * taken with x2 ln|x| as its logarithmic term (the expansion of
 * d/dx2 H0(k|x|)).  x: device float64 [T][2]; out: device complex [T][2] =
 * (dG/dx1, dG/dx2) per target, in the plan's precision; flags as for qpgf_g2d
 * (1: within lattice_rmin of a lattice point, 2: far branch, 4: beyond the far
 * slab, 8: non-finite input; the flagged results are NaN).  Ownership: the
 * caller owns x, out and flags; the call is stream-ordered on the plan's stream.
 * Errors: QPGF_E_ARG for a plan of another kind, T < 0 or NULL pointers with
 * T > 0; QPGF_E_WOOD for excluded instances (before any launch). */
qpgf_status qpgf_g2d_grad(qpgf_plan* plan, double k, double alpha,
                          const double* x, int64_t T, void* out, uint8_t* flags);

/* Differences of second derivatives of the 2D G for two wavenumbers (Section 2.4.2),
 * plan of kind QPGF_KIND_G2D_HESS_DIFF: per target the three values
 * d_p d_q G_{k1}(x) - d_p d_q G_{k2}(x), pq = 11, 12, 22, with one alpha.  The
 * plan's three fields hold T_pq - h_pq, T_pq = e^{-i alpha x1} times that difference
 * (coefficients m_pq (K-hat^{(k1)}_j - K-hat^{(k2)}_j) - H-hat_pq,j with
 * m = -(alpha + j1)^2, -(alpha + j1) j2 pi/c~, -(j2 pi/c~)^2; the k-independent
 * 1/|x|^2 singularities cancel in the difference and the remaining singular parts
 * h_pq, of the logarithm and x_p x_q/|x|^2, come from the plan's tables).  h_pq is
 * taken with the constant +(k1^2 - k2^2)/(2 pi) (the expansion of the difference of
 * the two Hankel functions; the printed definitions carry a minus sign).  The far
 * slab holds the series (1.2) differentiated twice term by term.  x: device float64
 * [T][2]; out: device complex [T][3] (11, 12, 22) in the plan's precision; flags as
 * for qpgf_g2d.  k1 = k2 gives zeros.  Errors as for qpgf_g2d_grad, Wood checks for
 * both wavenumbers. */
qpgf_status qpgf_g2d_hess_diff(qpgf_plan* plan, double k1, double k2, double alpha,
                               const double* x, int64_t T, void* out, uint8_t* flags);

/* Preparation alone (stage 0: coefficients; 1: after the transverse transform; 2:
 * grids and far slab, ready for qpgf_evaluate) for a plan of kind
 * QPGF_KIND_G2D_HESS_DIFF, which qpgf_prepare and qpgf_prepare_stage refuse
 * (QPGF_E_ARG) because it needs two wavenumbers. */
qpgf_status qpgf_prepare_hess_diff(qpgf_plan* plan, double k1, double k2, double alpha, int stage);

/* Batched form of Algorithm 2.1: n_inst independent instances in one call.
 * Instance i has wavenumber k[i], alpha[i] and x1 size m1[i] (2^a r with a >= 1
 * and r in {1, 3, 5, 7}, 16 <= m1[i] <= params.m1; every instance uses the plan's transverse size m2
 * and method parameters) and owns targets t_off[i] .. t_off[i+1]-1 of the
 * concatenated device array x [t_off[n_inst]][2]; its results go to the same
 * positions of out (and flags).  k, alpha, m1 and t_off are HOST arrays, read
 * during the call.  Each stage (coefficient fill, transverse FFT, x1 FFT, far
 * slab, gather) is a single launch over all instances; the whole sequence is
 * captured once in a HIP graph and replayed on later calls with the same n_inst,
 * m1[], t_off[], x, out and flags (k and alpha may differ).  The 2D singular
 * tables of the plan serve every instance (they depend on the coefficient index
 * only, Remark 2.1).  Needs a plan of kind QPGF_KIND_G2D; every instance is
 * checked for Wood anomalies before any launch. */
qpgf_status qpgf_g2d_batched(qpgf_plan* plan, int n_inst, const double* k, const double* alpha, const int* m1,
                             const int64_t* t_off, const double* x, void* out, uint8_t* flags);

/* Caller-owned workspace.  A plan's bulk device arrays are the near grid (every
 * field), its node-interleaved copy (2D derivative kinds and the complex64 2D
 * G), the far slab (its size grows with the wavenumber: see far_m1, far_m2 and
 * the slab geometry in qpgf_plan_info) and the per-call target scratch (the
 * binning of 3D targets, the ring mask of 2D ring_interp).  By default the plan
 * allocates them itself and grows the slab and the scratch on demand.
 *
 * qpgf_plan_workspace_bytes: the bytes (in *bytes) of one device buffer that
 * holds all of them for instances of wavenumber up to kmax (both wavenumbers of
 * the second-derivative differences) and calls of up to max_targets targets.
 *
 * qpgf_plan_set_workspace: the plan frees its own arrays and lays them out in
 * [ptr, ptr + bytes) (device memory, 256-byte aligned, bytes at least what
 * qpgf_plan_workspace_bytes returns for the same kmax and max_targets).  From
 * then on no single-instance call allocates device memory: a prepare, g2d,
 * gd3d, maxwell3d, ... of a larger wavenumber, or an evaluate of more targets,
 * returns QPGF_E_SIZE instead.  The caller keeps the buffer alive and leaves it
 * alone until the plan is destroyed or given another workspace.  ptr = NULL
 * (bytes 0) returns the plan to allocating its own arrays.  Either way the grids
 * are lost: prepare again before evaluating.  Synchronises the plan's stream.
 * Not covered: the plan's constant tables, allocated at creation (quadrature,
 * twiddles, the 2D singular-part tables, and the 3D H table, sized for
 * |alpha_i| <= 1: an instance with a larger |alpha_i| grows it), the batched 2D
 * call's per-batch buffers, and the autotuner's scratch.  Errors: E_ARG (NULL plan or bytes, kmax not finite
 * or < 0, max_targets outside [0, 2^31 - 1], ptr not aligned), E_SIZE (bytes
 * too small), E_HIP / E_NOMEM (returning to the plan's own arrays). */
qpgf_status qpgf_plan_workspace_bytes(const qpgf_plan* plan, double kmax, int64_t max_targets, size_t* bytes);
qpgf_status qpgf_plan_set_workspace(qpgf_plan* plan, void* ptr, size_t bytes, double kmax, int64_t max_targets);

/* FFT autotuner: for every transform shape the plan uses (and, for 2D plans,
 * every power-of-two x1 length from 16 to params.m1, and params.m1), time the candidate numbers
 * of transforms per block on scratch memory and keep the fastest.  Results are
 * cached in the text file cache_path (NULL: no file), one line per shape:
 * "<arch> <prec> <n> <rows|cols> <batch> <tile> <us>"; shapes found there are not
 * re-timed.  Synchronous; call after plan creation. */
qpgf_status qpgf_plan_autotune(qpgf_plan* plan, const char* cache_path);

/* The interpolated smooth part L_N(t) of Algorithm 3.1 step 2d (K_d minus the
 * singular part F, without the phase) at T targets of the last prepared GD3D
 * instance; NaN for far targets (|x3| > c).  out: device complex [T] in the plan
 * precision.  Training data for the surrogate below. */
qpgf_status qpgf_evaluate_smooth(qpgf_plan* plan, const double* x, int64_t T, void* out);

/* MLP surrogate of the smooth part L_d(x; k, alpha1, alpha2) of G_d in the near
 * region |x3| <= 0.6 (c = 0.6, c~ = 1).  Architecture: 64 input features of
 * (x1, x2, x3, k, alpha1, alpha2) (harmonics of the reduced coordinates and of
 * k x, alpha x), four hidden layers of 256 with GELU, a 2-output head (Re, Im of
 * 10 L_d).  Hidden layers run on the matrix cores with bf16 operands and fp32
 * accumulation; parameters, gradients and Adam moments are fp32.  `members`
 * independently initialised networks form an ensemble whose spread is the error
 * estimate.  Queries q are device float64 [B][6] rows (x1, x2, x3, k, alpha1,
 * alpha2).  Parameters are a flat float32 vector of qpgf_mlp_param_count()
 * entries per member: W0 [256][64], b0, W1 [256][256], b1, W2, b2, W3, b3,
 * W4 [2][256], b4 (row-major; layer l computes z = W a + b). */
typedef struct qpgf_mlp qpgf_mlp;
long qpgf_mlp_param_count(void);
qpgf_status qpgf_mlp_create(int members, int64_t max_batch, uint64_t seed, qpgf_mlp** out);
void qpgf_mlp_destroy(qpgf_mlp* m);
qpgf_status qpgf_mlp_set_stream(qpgf_mlp* m, void* hip_stream);
qpgf_status qpgf_mlp_get_params(qpgf_mlp* m, int member, float* dst);       /* device [param_count] */
qpgf_status qpgf_mlp_set_params(qpgf_mlp* m, int member, const float* src); /* device [param_count] */
/* y: device float32 [B][2], the network output (10 L_d) for member `member`. */
qpgf_status qpgf_mlp_forward(qpgf_mlp* m, int member, const double* q, int64_t B, float* y);
/* Gradient of 0.5 mean_b |net(q_b) - y_b|^2 into grad (device [param_count]) and the
 * loss into loss (device float, may be NULL); B a multiple of 64, <= max_batch. */
qpgf_status qpgf_mlp_gradient(qpgf_mlp* m, int member, const double* q, const float* y, int64_t B, float* grad,
                              float* loss);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) on that loss. */
qpgf_status qpgf_mlp_train_step(qpgf_mlp* m, int member, const double* q, const float* y, int64_t B, float lr,
                                float* loss);
const char* qpgf_mlp_last_error(void);
/* The error estimate of the surrogate is the ensemble spread s (largest distance
 * of a member's L_d from the mean) times a calibration factor kappa fitted
 * against the plain method: a value is accepted only if kappa s <= tol |G_d|.
 * A new model has kappa = +inf and accepts nothing until calibrated (or until
 * a checkpoint with a finite kappa is loaded); kappa is not applied to models
 * of one member, which accept nothing.  set: kappa > 0 (+inf allowed). */
qpgf_status qpgf_mlp_set_calibration(qpgf_mlp* m, double kappa);
qpgf_status qpgf_mlp_get_calibration(const qpgf_mlp* m, double* kappa);
/* Training rows from the plain method: for instance i (host k, a1, a2, t_off as
 * in qpgf_g2d_batched) prepare `plan` (GD3D, c = 0.6, c~ = 1) and evaluate the
 * interpolated smooth part L_N (qpgf_evaluate_smooth) at device targets
 * x[t_off[i]..t_off[i+1])[3]; write q (device float64 [T][6]: x, k, alpha1,
 * alpha2) and y (device float32 [T][2]: 10 Re L_N, 10 Im L_N).  Runs on the
 * model's stream and synchronises it.  Errors: E_ARG, E_WOOD (the message
 * names the instance), E_SIZE, E_HIP/E_NOMEM. */
qpgf_status qpgf_surrogate_make_data(qpgf_mlp* m, qpgf_plan* plan, int n_inst, const double* k, const double* a1,
                                     const double* a2, const int64_t* t_off, const double* x, double* q, float* y);
typedef struct qpgf_train_cfg {
  int64_t batch;     /* rows per Adam step: a multiple of 64, <= the model's max_batch */
  int64_t steps;     /* Adam steps per member */
  float lr_max;      /* cosine schedule: lr_min + (lr_max - lr_min)(1 + cos(pi t / steps)) / 2 */
  float lr_min;
  int32_t member;    /* the member to train, or -1 for every member in turn */
  int32_t reserved;  /* 0 */
  uint64_t seed;     /* data order: a fresh shuffle of the N rows per epoch, per member */
} qpgf_train_cfg;
/* Adam on the squared loss over device rows q [N][6], y [N][2] (as written by
 * qpgf_surrogate_make_data), minibatches drawn without replacement.  The Adam
 * step counts continue from the model's (so a loaded checkpoint resumes).
 * loss: device float32 [members] or NULL, the last minibatch's loss of each
 * trained member.  Synchronises the model's stream before returning. */
qpgf_status qpgf_surrogate_train(qpgf_mlp* m, const double* q, const float* y, int64_t N, const qpgf_train_cfg* cfg,
                                 float* loss);
/* Fit kappa on held-out instances: for every near target (|x3| <= 0.6) of
 * instance i the ratio |L_mean - L_N| / s against the plain method's smooth
 * part of `plan`; kappa = safety times the `quantile` (0 < quantile <= 1; 1 =
 * the largest) of those ratios, stored in the model and returned in *kappa
 * (host, may be NULL).  Needs at least two members.  Allocates its scratch
 * (T complex values and T doubles).  Errors as qpgf_surrogate_make_data. */
qpgf_status qpgf_surrogate_calibrate(qpgf_mlp* m, qpgf_plan* plan, int n_inst, const double* k, const double* a1,
                                     const double* a2, const int64_t* t_off, const double* x, double quantile,
                                     double safety, double* kappa);
/* Checkpoints: every member's float32 parameters, both Adam moments and step
 * count, and kappa, in one binary file ("QPGFMLP1", int32 members, int64
 * param_count, float64 kappa, then per member int64 step and 3 param_count
 * float32: parameters, first moment, second moment; little-endian).  load
 * requires a file of a model with the same number of members and leaves the
 * model unchanged when the file is not such a checkpoint (E_IO). */
qpgf_status qpgf_mlp_save(qpgf_mlp* m, const char* path);
qpgf_status qpgf_mlp_load(qpgf_mlp* m, const char* path);
/* G_d from the surrogate for n_inst instances (host k, a1, a2, t_off as in
 * qpgf_g2d_batched; device targets x [t_off[n]][3]) with fallback: a target takes
 * the plain method (the GD3D plan `plan`, whose precision sets out's type) when it
 * is far (|x3| > 0.6, flag 2), when the calibrated error estimate exceeds tol
 * |G_d| or the model is uncalibrated (flag 4), when its instance is within
 * wood_tol of a Wood anomaly (flag 8), or within
 * rmin of a lattice point (flag 16).  fell_back: device uint8 [T] of those flags
 * (0 = surrogate value); *n_fallback (host, may be NULL) receives their count.
 * Synchronises the model's stream once (to size the fallback work) and sets the
 * plan's stream to the model's.  Errors: E_ARG (NULLs, plan not GD3D or not
 * c = 0.6, c~ = 1), E_WOOD from the plain method on a fallback instance
 * (message names the instance), E_HIP/E_NOMEM. */
qpgf_status qpgf_surrogate_eval(qpgf_mlp* m, qpgf_plan* plan, double tol, double wood_tol, double rmin, int n_inst,
                                const double* k, const double* a1, const double* a2, const int64_t* t_off,
                                const double* x, void* out, uint8_t* fell_back, int64_t* n_fallback);

/* Stage outputs for parity checks.  qpgf_prepare_stage runs the preparation only
 * up to `stage`: 0 = coefficient fill (A L-hat_j with A the basis normalisation
 * 1/(2 sqrt(pi c~)) in 2D, 1/sqrt(8 pi^2 c~) in 3D, in FFT order: index j mod m
 * per axis), 1 = after the transverse inverse FFT, 2 = complete near grid
 * L_N(x_p) (grid point p mod m per axis, x = p h) and far slab.  qpgf_copy_field
 * copies field `field` of the near grid buffer (which = 0; 0 = L, then L^{pq} in
 * the order 11,22,33,12,13,23, without 33 under maxwell_trace) or of the far slab
 * (which = 1; info.far_fields fields) to the device pointer dst, which must hold
 * info.grid_bytes / info.far_grid_bytes.  Layout: [i3][i2][i1] (3D) or [i2][i1]
 * (2D) with i1 fastest; far slab: [s][i2][i1] or [s][i1] on its own far_m1 x far_m2
 * periodic grid, slice s at |x_t| = c - 3 h_f + s h_f; a far-slab value times
 * e^{i alpha.x'} is the series (G, G_d or GG_pq) at that node. */
qpgf_status qpgf_prepare_stage(qpgf_plan* plan, double k, double a1, double a2, int stage);
qpgf_status qpgf_copy_field(qpgf_plan* plan, int which, int field, void* dst);

/* Per-kernel timing, for profiling.  While enabled, every kernel the plan
 * launches is bracketed by HIP events recorded on the plan's stream (the stream
 * the kernel runs on).  qpgf_plan_get_timing waits for the recorded events and
 * returns, for kernel class `id`, the summed duration in milliseconds and the
 * number of launches since timing was last enabled.  Enabling resets the sums.
 * Classes: */
typedef enum {
  QPGF_T_HTABLE = 0,   /* radial table H(rho) of the 3D singular transform       */
  QPGF_T_FILL = 1,     /* FP64 coefficient fill of the near fields               */
  QPGF_T_FFT_T = 2,    /* inverse FFT along the transverse axis                  */
  QPGF_T_FFT_2 = 3,    /* inverse FFT along x2 (3D)                              */
  QPGF_T_FFT_1 = 4,    /* inverse FFT along x1                                   */
  QPGF_T_FAR = 5,      /* far-slab coefficient fill                              */
  QPGF_T_FAR_FFT = 6,  /* inverse FFTs of the far slab                           */
  QPGF_T_GATHER = 7,   /* interpolation gather, add-back and phase               */
  QPGF_T_BIN = 8,      /* target binning by grid tile: counts and offset scans   */
  QPGF_T_BATCH = 9,    /* one replay of the batched 2D graph (all stages)        */
  QPGF_T_BIN_PLACE = 10, /* binning: scatter of target records into tile order   */
  QPGF_T_OVERFLOW = 11,  /* targets handed over by the tiled gather              */
  QPGF_T_LAYOUT = 12,    /* 2D: derivative fields interleaved per node, or the     */
                         /* complex64 G's node quads (4 x1-neighbours per node)  */
  QPGF_T_RING = 13,      /* 2D kinds with ring_interp: the cut-off-ring correction */
  QPGF_T_GATHER_FAR = 14,  /* 3D binned calls: the far-tile gather (QPGF_T_GATHER: near tiles) */
  QPGF_T_COUNT = 15
} qpgf_timer_id;
qpgf_status qpgf_plan_enable_timing(qpgf_plan* plan, int on);
qpgf_status qpgf_plan_get_timing(qpgf_plan* plan, int id, double* total_ms, int64_t* launches);

/* Message for the last error on the calling thread ("" if none). */
const char* qpgf_last_error(void);

/* Library version string. */
const char* qpgf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* QPGF_H */
