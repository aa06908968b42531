/*
 * isdf_xtc.h -- C ABI of libisdfxtc, the MI355X (gfx950) implementation of the
 * data-parallel hot path of ISDF-xTC (arXiv 2607.17314): orbital values on a
 * real-space grid, ISDF interpolation-point selection and fit, and the
 * ISDF-compressed transcorrelated two-body intermediates built from grid-pair
 * kernel tiles that are generated on the fly and never stored.
 *
 * Conventions shared by every call
 *  - Plain C99 types only. "device" pointers are HIP device memory, "host"
 *    pointers are host memory. Arrays are dense and row-major in the order the
 *    brackets give, the last index fastest; every device array must be 8-byte
 *    aligned (256-byte alignment is recommended).
 *  - Ownership: the caller owns every buffer. The library allocates no device
 *    memory: all scratch comes from the caller's workspace (ws, ws_bytes),
 *    whose required size xtc_workspace_bytes() returns for the same arguments.
 *  - Streams: `stream` is a hipStream_t (NULL = the default stream). Work is
 *    enqueued on it; calls with host outputs synchronise it before returning.
 *  - Errors: arguments are checked before anything is launched. A negative
 *    status is an error (outputs undefined); a positive status is a warning
 *    (outputs valid, see the code). xtc_last_error() returns a thread-local
 *    message for the last failing call on the calling thread.
 *  - Weights: every call that takes an xtc_grid and a workspace first checks on
 *    the device that the weights are finite and non-negative (one small kernel
 *    writing an integer flag into the first bytes of ws), synchronises the stream
 *    to read the flag, and returns XTC_ERR_INVALID_ARG before any other launch if
 *    one is not.
 *  - Determinism: reductions use fixed trees and no floating-point atomics,
 *    so repeated calls on the same inputs give bitwise-identical results.
 *  - Units: bohr for coordinates, hartree-scale quantities in FP64.
 */
#ifndef ISDF_XTC_H
#define ISDF_XTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t xtc_status;
enum {
  XTC_OK = 0,
  XTC_WARN_RANK_DEFICIENT = 1, /* fewer pivots than asked: residual exhausted */
  XTC_WARN_JITTER = 2,         /* a Tikhonov shift was needed in the fit */
  XTC_WARN_FALLBACK = 3,       /* learned points rejected, QR pivots returned */
  XTC_ERR_INVALID_ARG = -1,
  XTC_ERR_NOT_SPD = -2,        /* Gram matrix not SPD after the last shift */
  XTC_ERR_HIP = -3,            /* HIP runtime error; message in xtc_last_error */
  XTC_ERR_NO_WORKSPACE = -4,   /* ws_bytes below the requirement */
  XTC_ERR_UNSUPPORTED = -5
};

/* Arithmetic of the grid-pair contraction (xtc_kernel_contract, xtc_grad), and the
 * storage type of the interpolation vectors xi (isdf_fit's xi_prec, xtc_xi_source). */
enum {
  XTC_FP64 = 0,      /* FP64 kernels and FP64 MFMA throughout */
  XTC_FP32 = 1,      /* storage of xi only: FP32 (half the memory; the split path reads it) */
  XTC_SPLIT_F16 = 2  /* stage 1 as FP16 hi+lo split products on MFMA with FP32
                        accumulation and FP64 compensation across ket chunks;
                        stage 2, Gram/Cholesky and energy-scale sums in FP64 */
};

/* Correlator forms (Jastrow correlator section, eqs. bh-scaled and bh-u). */
enum {
  XTC_U_EE = 0, /* u = sum_k c_k rbar12^{o_k}, rbar = d r/(1 + d r) */
  XTC_U_BH = 1  /* multi-centre Boys-Handy form of eq. bh-u */
};

/* Channels of xtc_kernel_contract (bit mask). */
enum {
  XTC_U1 = 1,      /* u1[c][mu][nu] = sum_{g,g'} w w' xi~^c_mu(g) xi_nu(g') d_c u(g,g') (eq. K1-isdf) */
  XTC_U3 = 2,      /* u3[mu][nu]   = sum w w' xi_mu(g) xi_nu(g') |grad_1 u|^2 (eq. K3-isdf) */
  XTC_ULAP = 4,    /* ulap[mu][nu] = sum w w' xi_mu(g) xi_nu(g') lap_1 u (validation; EE only) */
  XTC_D1 = 8,      /* D1 = sum_g w xi_mu(g) V_nu(g) (xTC Term 1) */
  XTC_D4 = 16,     /* D4 = sum_g wt_g sum_c calG^c_mu calG^c_nu (xTC Term 4) */
  XTC_FIELD = 32,  /* field[c][g] = A_gamma^c(g) = sum_g' w' rho(g') d_c u(g,g') (exact) */
  XTC_ESCALE = 64  /* escale[6] energy-scale scalars, see xtc_kernel_contract */
};

/* Modes of isdf_select_points. */
enum {
  XTC_SELECT_QR = 0,            /* weight-scaled pivoted Cholesky (Alg. 1), both channels, fused */
  XTC_SELECT_LEARNED = 1,       /* MLP proposal + restricted pivoting, no judge */
  XTC_SELECT_LEARNED_JUDGED = 2 /* as 1, then fall back to QR if the fit residual exceeds
                                   fallback_factor times the QR residual */
};

/* Fit outputs of isdf_fit (bit mask). */
enum { XTC_FIT_XI = 1, XTC_FIT_XIGRAD = 2, XTC_FIT_KEEP_CHOL = 4 };

/* Doubles of one system's kept factor (isdf_fit with XTC_FIT_KEEP_CHOL): the lower
 * Cholesky factor L of A + shift I, row-major n_mu x n_mu (its strict upper triangle
 * unspecified), then the inverses of its 64 x 64 diagonal blocks [ceil(n_mu / 64)][64][64]
 * (the last block zero-padded), as the blocked triangular solves use them. */
#define XTC_CHOL_SYSTEM_DOUBLES(n_mu) \
  ((size_t)(n_mu) * (size_t)(n_mu) + (size_t)4096 * (size_t)(((n_mu) + 63) / 64))

/* Integration grid. */
typedef struct {
  int64_t n_g;
  const double* xyz; /* device [3][n_g] (SoA), bohr */
  const double* w;   /* device [n_g], quadrature weights, w >= 0 */
} xtc_grid;

/* Cartesian Gaussian basis (all arrays host; copied into the workspace).
 * chi_a(r) = comp_factor[a] x^i y^j z^k sum_p prim_coef[p] exp(-prim_exp[p] |r-R|^2),
 * (x,y,z) = r - atom_xyz[shell_center[s]], p over the primitives of the AO's shell s.
 * AOs are shell-major; a shell of angular momentum l holds (l+1)(l+2)/2 AOs with
 * (i,j,k), i+j+k = l, i descending, then j descending. */
typedef struct {
  int32_t n_atom;
  const double* atom_xyz;          /* host [n_atom][3] */
  int32_t n_shell;
  const int32_t* shell_center;     /* host [n_shell] */
  const int32_t* shell_l;          /* host [n_shell], 0 <= l <= 6 */
  const int32_t* shell_prim_start; /* host [n_shell + 1] */
  const double* prim_exp;          /* host [n_prim] */
  const double* prim_coef;         /* host [n_prim] */
  const double* comp_factor;       /* host [n_ao] */
  int32_t n_ao;
} xtc_basis;

/* Correlator (all arrays host). EE: n_types = 1, mno[k] = (0, 0, o_k).
 * BH: u = sum_I sum_k c[type(I)][k] [a_1I^m a_2I^n + a_2I^m a_1I^n] rbar12^o,
 * a_iI = b[type(I)] r_iI / (1 + b[type(I)] r_iI). */
typedef struct {
  int32_t form;            /* XTC_U_EE or XTC_U_BH */
  int32_t n_terms;
  const int32_t* mno;      /* host [n_terms][3] */
  int32_t n_types;
  const double* c;         /* host [n_types][n_terms]: the linear coefficients */
  double d;                /* electron-electron scale, d > 0 */
  const double* b;         /* host [n_types] (BH only) */
  int32_t n_nuc;
  const double* nuc_xyz;   /* host [n_nuc][3] (BH only) */
  const int32_t* nuc_type; /* host [n_nuc] (BH only) */
} xtc_correlator;

/* Learned point scorer (not part of the paper; see isdf_select_points):
 * MLP 8 -> hidden -> hidden -> 1 with SiLU on z-scored log features, FP32 weights
 * packed as W1[hidden][8], b1[hidden], W2[hidden][hidden], b2[hidden], W3[hidden], b3. */
typedef struct {
  int32_t in_dim;          /* must be 8 */
  int32_t hidden;          /* 1 .. 128 */
  const float* params;     /* device, 8h + h + h*h + h + h + 1 floats */
  const float* feat_shift; /* device [8]: feature z-score shift */
  const float* feat_scale; /* device [8]: feature z-score scale */
  double kappa;            /* candidates by score = ceil(kappa * n_mu), clamped to n_g */
  int32_t n_nuc;           /* nuclei for the distance features */
  const double* nuc_xyz;   /* host [n_nuc][3] */
  int32_t judge;           /* 0: reference residual from the fit below; 1: run the QR
                              selection and use its residual (validation) */
  double ref_a, ref_b;     /* judge 0: log R_ref = ref_a + ref_b log(n_mu / n_orb) */
  int32_t stride;          /* coverage: every stride-th grid point is a candidate too (0: none) */
  int32_t bf16;            /* scoring: 0 FP32 on the vector units; 1 BF16 matrix cores (MFMA,
                              FP32 accumulation; hidden must be 64) */
} xtc_mlp;

/* Exchange intermediates requested from xtc_kernel_contract (xTC Terms 2 and 3,
 * see xtc_exchange_terms for the definitions): the orbitals at the pivots, the
 * projector gamma = lq lq^T and the outputs. All pointers are device memory. */
typedef struct {
  int32_t n_orb;
  const double* phi_piv; /* [n_orb][n_mu] */
  int32_t n_q;           /* projector rank, 1..32 */
  const double* lq;      /* [n_orb][n_q] */
  double* X2;            /* [n_orb][n_orb][n_mu] or NULL */
  double* X3;            /* [n_orb][n_orb][n_mu] or NULL */
} xtc_exchange;

/* Inputs of the four-index assembly (xtc_assembly_prepare, xtc_assembly_panel,
 * xtc_one_body): the orbitals at the pivots and the ISDF intermediates of
 * xtc_kernel_contract and xtc_exchange_terms. All pointers are device memory. */
typedef struct {
  int32_t n_orb, n_mu;
  const double* phi4_piv; /* [4][n_orb][n_mu]: phi_p and d_c phi_p at the pivots */
  const double* u1;       /* [3][n_mu][n_mu] */
  const double* u3;       /* [n_mu][n_mu] */
  const double* D1;       /* [n_mu][n_mu] */
  const double* D4;       /* [n_mu][n_mu] */
  const double* X2;       /* [n_orb][n_orb][n_mu] or NULL (taken as zero) */
  const double* X3;       /* [n_orb][n_orb][n_mu] or NULL (taken as zero) */
} xtc_assembly;

/* Outputs of the four-index assembly (bit mask). */
enum { XTC_ASM_K = 1, XTC_ASM_DU = 2, XTC_ASM_W = 4 };

/* Thread-local message of the last failing call (valid until the next call). */
const char* xtc_last_error(void);

/* Library version string. */
const char* xtc_version(void);

/* Call identifiers for xtc_workspace_bytes. */
enum { XTC_CALL_EVAL_ORBITALS = 1, XTC_CALL_SELECT = 2, XTC_CALL_FIT = 3,
       XTC_CALL_CONTRACT = 4, XTC_CALL_GRAD = 5, XTC_CALL_FEATURES = 6, XTC_CALL_MLP_GRAD = 7,
       XTC_CALL_EXCHANGE = 8, XTC_CALL_ASSEMBLY = 9, XTC_CALL_ONE_BODY = 10, XTC_CALL_VMC = 11 };

/* Flag of the contraction's workspace query: xi~ formed per bra super-block. */
#define XTC_WS_XIGRAD_BLOCKS (1u << 24)
/* Flag of the contraction's workspace query: the correlator is of the BH form (its pair
 * values are generated into a buffer of the workspace, in either precision). */
#define XTC_WS_BH (1u << 25)

/* Workspace bytes a call needs. flags: channels (CONTRACT/GRAD, with the
 * precision in bits 16..23 and, for CONTRACT, XTC_WS_XIGRAD_BLOCKS and XTC_WS_BH) or the
 * select mode
 * (SELECT) or the fit mask (FIT) or
 * the precision (EXCHANGE) or the output mask (ASSEMBLY; ONE_BODY takes none); for
 * SELECT in a learned mode, flags = mode | (mlp->stride << 8) and n_aux = ceil(100 kappa).
 * n_aux: n_ao (EVAL_ORBITALS, VMC), n_params (GRAD), the
 * projector rank n_q (EXCHANGE, and CONTRACT with exchange outputs, where n_aux > 0
 * asks for them), else 0. n_orb: the orbitals (also for CONTRACT with exchange outputs or
 * XTC_WS_XIGRAD_BLOCKS). */
size_t xtc_workspace_bytes(int32_t call, int64_t n_g, int32_t n_orb, int32_t n_mu,
                           int32_t n_aux, uint32_t flags);

/* Orbital and orbital-gradient values on the grid (Alg. 2, grid step):
 * phi4[0][p][g] = phi_p(r_g), phi4[1+c][p][g] = d_c phi_p(r_g), phi_p = sum_a chi_a C_mo[a][p].
 * C_mo: device [n_ao][n_orb]. phi4: device [4][n_orb][n_g] (output).
 * rho: device [n_g] or NULL; receives rho_gamma(g) = sum_{i < n_occ} phi_i(g)^2
 * (one-spin reference density, xTC section eq. deltaU-fields). Asynchronous. */
xtc_status xtc_eval_orbitals(const xtc_basis* basis, const xtc_grid* grid, const double* C_mo,
                             int32_t n_orb, int32_t n_occ, double* phi4, double* rho,
                             void* ws, size_t ws_bytes, void* stream);

/* Interpolation-point selection (ISDF section, pivot selection and fusion; Alg. 1).
 * Learned modes (not in the paper): score every point with the MLP; the candidates are
 * the ceil(kappa n_mu) best (ties to the lowest index) and every mlp->stride-th grid
 * point (coverage of the whole grid); the same fused pivoting runs restricted to the
 * candidates; XTC_SELECT_LEARNED_JUDGED then computes R, the mean of the four relative
 * weighted fit residuals (scalar and the three gradient components, as isdf_fit reports
 * them) of the proposal over the whole grid, and falls back to the QR selection
 * (XTC_WARN_FALLBACK) when R > fallback_factor R_ref.
 * QR mode: matrix-free weight-scaled pivoted Cholesky, FP64, on the scalar channel
 * d_g = w_g^2 (sum_p phi_p^2)^2 and the gradient channel
 * d_g = w_g^2 (sum_p phi_p^2)(sum_{p,c} (d_c phi_p)^2); ties go to the lowest index;
 * fused by fill-to-target: gradient channel to ceil(n_mu/2) pivots, then the scalar
 * channel extended until the union holds n_mu points; output order = scalar pivots in
 * selection order, then gradient-only pivots. Stops early (XTC_WARN_RANK_DEFICIENT)
 * when max_g d_g <= 1e-14 max_g D_g.
 * phi4: device [4][n_orb][n_g]. pivots: host [n_mu_target] (output), *n_mu_out: count.
 * info: host [8] or NULL: {scalar steps, gradient steps, used_fallback, R_selected,
 * R_qr (when computed), time_ms, candidates, 0}. mlp is required for the learned modes.
 * Synchronising. */
xtc_status isdf_select_points(const double* phi4, const xtc_grid* grid, int32_t n_orb,
                              int32_t n_occ, int32_t n_mu_target, int32_t mode,
                              const xtc_mlp* mlp, double fallback_factor, int64_t* pivots,
                              int32_t* n_mu_out, double* info, void* ws, size_t ws_bytes,
                              void* stream);

/* ISDF fit (ISDF section, eq. isdf-rho and its normal equations):
 * scalar A = G o G, G = Phi_mu^T Phi_mu; B = P o P, P = Phi_mu^T Phi; A xi = B.
 * gradient A_c = (dPhi_mu^T dPhi_mu)_c o G; B_c = P o (dPhi_mu^T dPhi)_c; A_c xi~^c = B_c.
 * Solved by FP64 Cholesky with the adaptive Tikhonov retry (no shift, then
 * 1e-14 * 10^k * mean(diag A), k = 0..8) and blocked triangular solves, in FP64 whatever
 * the storage type of xi. The grid is processed in chunks, each column on its own (the
 * fit is column-separable).
 * what: XTC_FIT_XI (xi), XTC_FIT_XIGRAD (xi~), XTC_FIT_KEEP_CHOL (the four factors to
 * chol, also those of systems whose solution is not asked for; the contraction forms xi~
 * per bra block from them when it is given no xigrad).
 * pivots: host [n_mu]. xi_prec: XTC_FP64 or XTC_FP32, the type of xi: device [n_mu][n_g]
 * (XTC_FP32: each element the rounding of the FP64 solution).
 * xigrad: device double [3][n_mu][n_g] (if what & XTC_FIT_XIGRAD).
 * chol: device double [4][XTC_CHOL_SYSTEM_DOUBLES(n_mu)] (if what & XTC_FIT_KEEP_CHOL):
 * scalar, x, y, z.
 * rho, rhot: device [n_g] each, or both NULL: with XTC_FIT_XI, rhot receives the ISDF
 * density rhot(g) = sum_mu rho(r_mu) xi_mu(g) (xTC section; rho the reference density)
 * from the FP64 solution, before any FP32 rounding of xi. That sum cancels heavily (xi
 * is large and sign-alternating where rhot is O(1)), so with FP32 xi the contraction
 * should take this rhot (xtc_xi_source) rather than re-forming it from the rounded xi.
 * info: host [8] or NULL: {shift index k per system (-1 none) x4, relative weighted
 * residual sum_g w^2 (|m_g|^2 - xi(g).B(g)) / sum_g w^2 |m_g|^2 x4} (scalar, x, y, z; the
 * residual of a system is reported when its solution is asked for, else 0).
 * Returns XTC_WARN_JITTER if any shift was used. Synchronising. Grids of more than 65,536
 * points run their column chunks on `stream` and up to two internal streams of the
 * library (per device, default priority), joined back into `stream` before it returns. */
xtc_status isdf_fit(const double* phi4, const xtc_grid* grid, int32_t n_orb,
                    const int64_t* pivots, int32_t n_mu, uint32_t what, int32_t xi_prec,
                    void* xi, double* xigrad, double* chol, const double* rho, double* rhot,
                    double* info, void* ws, size_t ws_bytes, void* stream);

/* Where xtc_kernel_contract takes xi and xi~ from, when not from the defaults (FP64 xi and
 * a stored xigrad): xi in FP32 (split path only), and xi~ formed per bra super-block
 * (xigrad = NULL with XTC_U1) from the orbitals and the fit's kept factors, with the fit's
 * own right-hand-side products and blocked solves for the block's columns (so the same
 * values as a stored xigrad, bit for bit, without its [3][n_mu][n_g] of memory). */
typedef struct {
  int32_t xi_prec;     /* XTC_FP64 or XTC_FP32: the element type of xi */
  const double* phi4;  /* device [4][n_orb][n_g], or NULL when xigrad is given */
  int32_t n_orb;
  const double* chol;  /* device: isdf_fit's kept factors [4][XTC_CHOL_SYSTEM_DOUBLES(n_mu)],
                          or NULL when xigrad is given */
  const double* rhot;  /* device [n_g]: the ISDF density from isdf_fit, or NULL to form it
                          from xi (recommended with FP32 xi, see isdf_fit) */
} xtc_xi_source;

/* Grid-pair kernels and xTC D terms, with the kernel tiles generated on the fly
 * (K-kernel section, eqs. K1-isdf and K3-isdf; xTC section Terms 1 and 4, with
 * calG^c_{mu,g} = sum_g' w_g' xi_mu(g') d_c u(g,g'), H_{g,c} = sum_l G_l calG^c_{l,g},
 * V_{nu,g} = sum_c H_{g,c} calG^c_{nu,g}, wt_g = w_g sum_l G_l xi_l(g), and
 * G_nu = rho_gamma(r_nu)). grad acts on the bra point g.
 * xi: device [n_mu][n_g] (FP64, or FP32 per src); xigrad: device [3][n_mu][n_g] (needed
 * for XTC_U1 unless src provides the factors).
 * rho: device [n_g] (rho_gamma). pivots: host [n_mu] (G is gathered from rho).
 * Outputs (device, FP64, overwritten; NULL when the channel is off):
 *   u1 [3][n_mu][n_mu], u3, ulap, D1, D4 [n_mu][n_mu], field [3][n_g].
 * escale: host [6] or NULL: {E3, E4, E1, E3x, E4x, E1x} with E3 = G^T u3 G,
 *   E4 = G^T D4 G, E1 = 2 G^T D1 G and their ISDF-free counterparts
 *   E3x = sum_{g,g'} w w' rho rho' |grad_1 u|^2, E4x = sum_g w rho |A_gamma|^2, E1x = 2 E4x.
 * precision: XTC_FP64 or XTC_SPLIT_F16. The BH form runs on both (without XTC_ULAP): the
 *   four channels of every grid pair are generated in FP64, one ket range of 16,384 points
 *   at a time, and stored for the products, split into FP16 pairs in split precision
 *   (workspace query with XTC_WS_BH: about bp x 256 KiB more, bp the super-block width of
 *   at most 16,384 points) or in FP64 (bp x 512 KiB more); its exchange outputs (ex) need
 *   XTC_FP64 (XTC_ERR_UNSUPPORTED otherwise).
 * [bra_begin, bra_end): the bra points g summed over (non-empty, inside the grid; the ket
 *   sums always cover the whole grid). (0, n_g) gives the outputs above; disjoint ranges
 *   give partial sums that add up to them (the bra sharding across devices); field is
 *   written for the range and zero elsewhere, and escale holds the range's partial sums.
 * ex: NULL, or the exchange intermediates X2, X3 of xTC Terms 2 and 3 to form in the
 *   same pass from the same calG panels (Alg. 2, xTC-correction step; definitions at
 *   xtc_exchange_terms); with ex the workspace query takes n_orb = ex->n_orb and
 *   n_aux = ex->n_q (FP64 xi only).
 * src: NULL (xi FP64; XTC_U1 needs xigrad), or the xi storage type and, for xigrad = NULL,
 *   the orbitals and kept factors (see xtc_xi_source); then the workspace query takes
 *   n_orb = src->n_orb and flags bit 24 (XTC_WS_XIGRAD_BLOCKS).
 * Asynchronous after the weight check; synchronising if escale != NULL. In split precision
 *   part of stage 2 runs on an internal stream of the library (one per device, created on
 *   first use, default priority), forked from and joined back into `stream` with events
 *   in each bra super-block: the call's work is complete when the work enqueued on
 *   `stream` is. */
xtc_status xtc_kernel_contract(const xtc_grid* grid, const xtc_correlator* corr, int32_t n_mu,
                               const void* xi, const double* xigrad, const double* rho,
                               const int64_t* pivots, uint32_t channels, int32_t precision,
                               int64_t bra_begin, int64_t bra_end, double* u1, double* u3,
                               double* ulap, double* D1, double* D4, double* field,
                               double* escale, const xtc_exchange* ex, const xtc_xi_source* src,
                               void* ws, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): xtc_kernel_contract without a
 * workspace. Same arguments, outputs and results as xtc_kernel_contract, minus ws and
 * ws_bytes. Its scratch is one file-scope device array of XTC_NOALLOC_SCRATCH_BYTES
 * bytes per device, which the library holds from the first call on that device until the
 * process ends; the call allocates and frees nothing. The bra super-blocks are narrowed
 * (halved, in multiples of 64 points) until the scratch fits, which only reorders the
 * stage-2 sums; with the regular call's width the results are bitwise those of
 * xtc_kernel_contract. A problem that needs more scratch even at 64-point super-blocks
 * (for example the split path's operand, 4 bytes per row and grid point) returns
 * XTC_ERR_NO_WORKSPACE. Every byte of the scratch that a call reads it has written
 * earlier in the same call, so contents left by an earlier call do not matter; calls
 * that overlap in time on one device (two host threads, or two streams) share the one
 * array and race: serialise them. */
#define XTC_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
xtc_status xtc_kernel_contract_noalloc(const xtc_grid* grid, const xtc_correlator* corr,
                                       int32_t n_mu, const void* xi, const double* xigrad,
                                       const double* rho, const int64_t* pivots, uint32_t channels,
                                       int32_t precision, int64_t bra_begin, int64_t bra_end,
                                       double* u1, double* u3, double* ulap, double* D1, double* D4,
                                       double* field, double* escale, const xtc_exchange* ex,
                                       const xtc_xi_source* src, void* stream);

/* Exchange intermediates of xTC Terms 2 and 3 through the low-rank projector
 * (xTC section, "Terms 2 and 3 (non-factorizable)", "Low-rank projector for Terms
 * 2 and 3"; pipeline section, symmetry paragraph). With gamma = LQ LQ^T,
 *   P[s a][nu]   = phi_s(r_nu) sum_t phi_t(r_nu) LQ[t][a],
 *   R^c[s a](g)  = sum_nu P[s a][nu] calG^c_{nu,g},   Q[s a](g) = sum_nu P[s a][nu] xi_nu(g),
 *   X2[q][s][mu] = sum_g w_g xi_mu(g) sum_{a,c} R^c[s a](g) R^c[q a](g),
 *   X3[q][s][mu] = sum_{g,c} w_g calG^c_{mu,g} sum_a (Q[s a] R^c[q a] + R^c[s a] Q[q a])(g),
 * so that Term2 = -sum_mu C^p_r(mu) X2[q][s][mu] and Term3 likewise with X3.
 * calG is regenerated per bra super-block from the grid-pair kernel tiles (as in
 * xtc_kernel_contract); only the q <= s half is computed and mirrored.
 * xi: device [n_mu][n_g]. phi_piv: device [n_orb][n_mu], phi_p at the pivots.
 * lq: device [n_orb][n_q], n_q = 1..32 (the projector; for a closed-shell
 * reference the occupied columns of the identity). X2, X3: device
 * [n_orb][n_orb][n_mu] (outputs, FP64, overwritten; either may be NULL).
 * precision: XTC_FP64, or XTC_SPLIT_F16 (stage 1 and the X products as split
 * FP16 MFMA products with FP64 accumulation across chunks; EE correlator only).
 * [bra_begin, bra_end): the bra points g summed over (0 <= begin <= end <= n_g; the
 * ket sum inside calG always covers the whole grid). (0, n_g) gives X; disjoint
 * ranges give partial sums that add up to X (the bra sharding across devices).
 * Workspace: xtc_workspace_bytes(XTC_CALL_EXCHANGE, n_g, n_orb, n_mu, n_q,
 * precision). Synchronising. */
xtc_status xtc_exchange_terms(const xtc_grid* grid, const xtc_correlator* corr, int32_t n_mu,
                              const double* xi, int32_t n_orb, const double* phi_piv,
                              int32_t n_q, const double* lq, int32_t precision,
                              int64_t bra_begin, int64_t bra_end, double* X2, double* X3,
                              void* ws, size_t ws_bytes, void* stream);

/* Four-index assembly of the two-body corrections (K-kernel section, eq.
 * K-recombine-final with eqs. K1-isdf and K3-isdf; xTC section, eq.
 * delta-u-dx-kernels and the final assembly; Hamiltonian assembly section):
 *   K  = 1/2 P12 [K1 - K1swap + K3],  K1swap^{pq}_{rs} = K1^{rs}_{pq},
 *   dU = -P12 [C (D4 + 2 D1) C - C (X2 + X3)],   W = -K + dU,
 * P12 T^{pq}_{rs} = T^{pq}_{rs} + T^{qp}_{sr}, C^p_r(mu) = phi_p phi_r (r_mu).
 * xtc_assembly_prepare forms the pair factors and their projections once into the
 * workspace (size: xtc_workspace_bytes(XTC_CALL_ASSEMBLY, 0, n_orb, n_mu, 0, outputs));
 * xtc_assembly_panel then writes, for p0 <= p < p1, the panels
 *   K, dU, W: device [p1 - p0][n_orb][n_orb][n_orb], element [p - p0][r][q][s] = T^{pq}_{rs}
 * (electron 1's pair (p, r) first, then electron 2's (q, s)); NULL where the output is
 * not in `outputs`. The panel call reads the prepared workspace: pass the same ws, the
 * same inputs and the same outputs mask, unchanged since the prepare call. Panels may
 * be computed in any order and repeated. FP64 MFMA throughout. Asynchronous. */
xtc_status xtc_assembly_prepare(const xtc_assembly* a, uint32_t outputs, void* ws,
                                size_t ws_bytes, void* stream);
xtc_status xtc_assembly_panel(const xtc_assembly* a, uint32_t outputs, int32_t p0, int32_t p1,
                              double* K, double* dU, double* W, void* ws, size_t ws_bytes,
                              void* stream);

/* xTC one-body pieces (Hamiltonian assembly section, eqs. xtc-deltah, xtc-fock,
 * xtc-const) from partial traces over the first n_occ (occupied) orbitals, without the
 * four-index tensors:
 *   dh_{pq} = -1/2 sum_o (2 dU^{po}_{qo} - dU^{po}_{oq}),
 *   f_{pq}  = dh_{pq} + sum_i (2 W^{pi}_{qi} - W^{pi}_{iq}),
 *   e0      = -2/3 sum_i dh_{ii} + e_nuc.
 * dh, f: device [n_orb][n_orb] or NULL; e0: host [1] or NULL (synchronising when set).
 * Workspace: xtc_workspace_bytes(XTC_CALL_ONE_BODY, 0, n_orb, n_mu, 0, 0). FP64. */
xtc_status xtc_one_body(const xtc_assembly* a, int32_t n_occ, double e_nuc, double* dh,
                        double* f, double* e0, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of xtc_kernel_contract with respect to the linear coefficients c:
 * dtheta[j] = dL/dc_j for L = sum_c <gu1_c, u1_c> + <gu3, u3> + <gulap, ulap>
 * + <gD1, D1> + <gD4, D4> + <gfield, field>. Cotangents: device, shapes of the
 * matching outputs, NULL when absent. Kernel tiles are regenerated, never stored;
 * the D cotangents add one recomputation pass of calG.
 * dtheta: device [n_types * n_terms] (output). dd: device or NULL; it receives the
 * derivatives with respect to the nonlinear parameters: for the EE form [1] = dL/dd
 * for the scale d of rbar = d r / (1 + d r); for the BH form [1 + n_types] =
 * dL/dd, then dL/db_t for the scale b_t of a_I = b r_I / (1 + b r_I) on the nuclei of
 * type t (eq. bh-u). Asking for dd leaves dtheta unchanged; for the BH form it runs a
 * separate kernel variant (more registers) so the dd = NULL path keeps its own.
 * [bra_begin, bra_end): the bra points of the outputs being differentiated, as for
 * xtc_kernel_contract (non-empty, inside the grid): the derivative of the range's partial
 * sums, so disjoint ranges give derivatives that add up to the whole grid's (0, n_g).
 * FP64. Asynchronous after the weight check (see the conventions). */
xtc_status xtc_grad(const xtc_grid* grid, const xtc_correlator* corr, int32_t n_mu,
                    const double* xi, const double* xigrad, const double* rho,
                    const int64_t* pivots, int64_t bra_begin, int64_t bra_end,
                    const double* gu1, const double* gu3,
                    const double* gulap, const double* gD1, const double* gD4,
                    const double* gfield, double* dtheta, double* dd, void* ws, size_t ws_bytes,
                    void* stream);

/* ---- Reference-variance VMC optimisation of the correlator (the VMC section) ----
 * Trial function Psi_T = F Phi_0 with F = prod_{i<j} exp(u(r_i, r_j)) (eq. tau-def) and
 * Phi_0 the closed-shell reference determinant over the n_occ occupied orbitals:
 * electrons 0 .. n_occ - 1 spin up, n_occ .. 2 n_occ - 1 spin down,
 * Phi_0 = det[phi_k(r_i)]_up det[phi_k(r_i)]_down. Hamiltonian: kinetic energy,
 * electron-nucleus attraction -Z_I / r_iI, electron repulsion 1 / r_ij and e_nuc.
 * Walkers: device [n_walkers][2 n_occ][3] FP64 (bohr). */
typedef struct {
  const xtc_basis* basis;   /* host tables, as for xtc_eval_orbitals */
  int32_t n_occ;            /* electrons per spin, 1 .. 32 */
  const double* C_occ;      /* device [n_ao][n_occ]: the occupied orbitals' coefficients */
  int32_t n_nuc;
  const double* nuc_xyz;    /* host [n_nuc][3] */
  const double* nuc_charge; /* host [n_nuc] */
  double e_nuc;             /* constant added to every local energy */
} xtc_vmc_system;

/* Metropolis sampling of |Phi_0|^2 (the VMC section samples the reference determinant,
 * not the trial function, so the draws do not depend on the correlator): n_sweeps
 * sweeps, each moving electrons 0 .. 2 n_occ - 1 in order with the symmetric proposal
 * r_i' = r_i + step * eta (product and sum rounded separately) and accepting when
 * uniform < |Phi_0(R') / Phi_0(R)|^2. The inverse Slater matrices are formed once per
 * call and kept by Sherman-Morrison updates.
 * R: device [n_walkers][2 n_occ][3], updated in place. normals: device
 * [n_sweeps][2 n_occ][n_walkers][3] standard normal draws; uniforms: device
 * [n_sweeps][2 n_occ][n_walkers] on [0, 1). accepted: device int64 [n_walkers], the
 * number of accepted moves, or -1 for a walker whose starting determinant is exactly
 * singular (left unmoved). With n_walkers = 0, R, accepted and the draws may be NULL.
 * Workspace: xtc_workspace_bytes(XTC_CALL_VMC, 0, 0, 0, n_ao, 0).
 * Limits: n_occ <= 32; per shell fewer than 32768 primitives, each starting below 32768,
 * and n_ao < 131072 (packed shell records); the walker's LDS within 160 KB: with n = n_occ,
 * 2 n^2 + max(2 n^2, 11 n) + n_ao + 6 n + 64 doubles and n ints, plus the basis tables
 * (4 per distinct shell centre + 2 n_prim doubles, 2 n_shell ints). FP64. Asynchronous
 * after the basis upload. */
xtc_status xtc_vmc_sample(const xtc_vmc_system* sys, int64_t n_walkers, double* R,
                          int32_t n_sweeps, double step, const double* normals,
                          const double* uniforms, int64_t* accepted, void* ws, size_t ws_bytes,
                          void* stream);

/* Local energies E_loc = H Psi_T / Psi_T (eq. Eloc) of the walkers R and, when dE is not
 * NULL, their derivatives in the correlator's parameters: for the EE form
 * u = sum_k c_k rbar^{o_k}, rbar = d r / (1 + d r), theta = (c_0 .. c_{n_terms - 1}, d);
 * for the BH form (eq. bh-u) theta = (c[type][term] type-major, d, b_0 .. b_{n_types - 1}):
 *   lap_i Psi_T / Psi_T = lap_i J + |grad_i J|^2 + 2 grad_i J . grad_i Phi_0 / Phi_0
 *                         + lap_i Phi_0 / Phi_0,  J = sum_{i<j} u(r_i, r_j).
 * E: device [n_walkers]; dE: device [n_walkers][number of parameters] or NULL. A walker
 * whose determinant is exactly singular gets NaN. EE: 1 .. 12 terms (0, 0, o). BH: 1 .. 24
 * nuclei, 1 .. 2 types, 1 .. 64 terms with m, n <= 3 and o <= 12, at most 128 parameters;
 * its linear derivatives are sums over electron pairs and nuclei of unit kernels, its d and
 * b derivatives are carried in forward mode. Workspace as xtc_vmc_sample; LDS per walker
 * within 160 KB, with n = n_occ and T the basis tables (as for xtc_vmc_sample): EE
 * 14 n^2 + 5 n_ao + 7 n + 384 doubles plus T; BH 12 n^2 + 15 n + 4 n_nuc + 704 doubles
 * plus the larger of (T + 2 n^2 + 5 n_ao + 320 doubles + n ints) and 12 n n_nuc doubles.
 * FP64. */
xtc_status xtc_vmc_local_energy(const xtc_vmc_system* sys, const xtc_correlator* corr,
                                int64_t n_walkers, const double* R, double* E, double* dE,
                                void* ws, size_t ws_bytes, void* stream);

/* One Newton step with Gauss-Newton curvature (eq. gn) on the fixed-batch clipped
 * variance (eq. var-loss): m = mean E, d = mean |E - m|, Et = clip(E, m - 5 d, m + 5 d),
 * r_k = Et_k - mean Et, sigma^2 = sum r_k^2 / (N - 1); the clipped energies' derivatives
 * follow the bounds m +- 5 d as functions of theta (sign(0) = 0 in d's derivative);
 * C = (1/N) sum_k dr_k dr_k^T + lambda I, delta = -eta C^-1 grad sigma^2 (Cholesky).
 * E: device [N]; dE: device [N][n_params] (1 .. 128 parameters); delta: device
 * [n_params]; stats: device [6] = m, d, mean Et, sigma^2, the number of clipped
 * energies, and 0 (or j + 1 when C's j-th pivot is not positive; delta is then NaN).
 * N >= 2. No workspace. FP64. Asynchronous. */
xtc_status xtc_vmc_gn_step(int64_t n_walkers, int32_t n_params, const double* E, const double* dE,
                           double lambda, double eta, double* delta, double* stats, void* stream);

/* Kernel timing for measurement: HIP events recorded on the call's stream around
 * each launch of the timed stages. mode 1: reset and start collecting; 0: stop and
 * reset; 2: synchronise the recorded events and write, per category c,
 * out[2c] = summed milliseconds and out[2c+1] = number of launches.
 * Categories: 0 stage 1 (pair kernel and density rows, per bra super-block),
 * 1 stage-2 GEMMs, 2 pivot selection, 3 fit, 4 orbitals, 5 adjoint pair kernel,
 * 6 MLP, 7 split-operand preparation, 8 the stage-1 pair kernel alone (one entry
 * per kernel launch), 9 exchange projections and pair products, 10 exchange X
 * products (operand splitting included), 11 the exchange's stage 1 on the projected
 * rows (split path), 12 the exchange's split X-product kernel alone (one entry per
 * launch), 13 the assembly panel kernel (one entry per launch), 14 VMC sampling,
 * 15 VMC local energies, 16 the Gauss-Newton step, 17 the pair-value generation of the BH
 * form in split precision (one entry per launch; its split products count under 8).
 * out: host [2 * XTC_TIMING_CATEGORIES]. Not thread-safe. */
#define XTC_TIMING_CATEGORIES 18
xtc_status xtc_timing(int32_t mode, double* out);

/* Learned-point features (see xtc_mlp): feats[k][g], k = 0..7 = log of w, sum phi^2,
 * sum (grad phi)^2, rho_gamma, |grad rho_gamma|, and the three smallest nuclear
 * distances (the last repeated if n_nuc < 3); log(x + 1e-30), computed in FP64.
 * phi4: device [4][n_orb][n_g]. nuc_xyz: host [n_nuc][3]. feats: device float [8][n_g]. */
xtc_status xtc_mlp_features(const double* phi4, const xtc_grid* grid, int32_t n_orb, int32_t n_occ,
                            int32_t n_nuc, const double* nuc_xyz, float* feats, void* ws,
                            size_t ws_bytes, void* stream);

/* MLP logits of n points: logits[i] = s(feats[:, i]) with the z-scoring of mlp; FP32, or
 * with mlp->bf16 the weights and activations rounded to BF16 on the matrix cores (FP32
 * accumulation, biases and SiLU in FP32). */
xtc_status xtc_mlp_forward(const xtc_mlp* mlp, const float* feats, int64_t ld, int64_t n,
                           float* logits, void* stream);

/* Weighted binary cross-entropy of n points (labels 0/1, float) and its gradient
 * w.r.t. the packed parameters: L = mean [pw y softplus(-s) + (1 - y) softplus(s)].
 * loss: device float [1]; grad: device float [n_params]. Deterministic. */
xtc_status xtc_mlp_loss_grad(const xtc_mlp* mlp, const float* feats, int64_t ld, int64_t n,
                             const float* labels, float pos_weight, float* loss, float* grad,
                             void* ws, size_t ws_bytes, void* stream);

/* One Adam step on device arrays (t = step number, from 1). */
xtc_status xtc_adam_step(float* params, const float* grad, float* m, float* v, int32_t n,
                         float lr, float beta1, float beta2, float eps, int32_t t, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* ISDF_XTC_H */
