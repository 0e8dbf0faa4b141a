/*
 * kp.h -- C ABI of the KSVD tensor-product block-Jacobi preconditioner for
 * very high order DG (Pazner & Persson, arXiv 1704.04549) on AMD MI355X.
 *
 * The preconditioner approximates each element's n^d x n^d diagonal block A_k
 * of M - tau*J (Sec. 3.4) by a short Kronecker sum of n x n factors
 * (eqs. 2d-kron-sum, 3d-simple-precond), found with the Van Loan rearrangement
 * and a top-r SVD computed by Lanczos (Sec. 4.1, Alg. 2), and inverts that sum
 * with sum-factorised n x n contractions plus a quasi-triangular Sylvester
 * solve (Sec. 4.2-4.4, Algs. 5-8).  n = p + 1 nodes per direction.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - All array arguments are DEVICE pointers unless the name ends in _h.
 * - The caller owns every buffer it passes; the library owns only the
 *   workspace held by a kp_ctx (the 1D tables of every n, built by kp_create;
 *   the rest allocated on first need, grown on demand, freed by kp_destroy)
 *   and the static scratch array of kp_setup_noalloc.
 * - Work is enqueued on the context's HIP stream; only kp_fgmres and
 *   kp_blockjacobi_exact synchronise (kp_fgmres once per Arnoldi step to read
 *   the Givens residual, or once per restart cycle under KP_OPT_FGMRES_GRAPHS;
 *   kp_blockjacobi_exact never except on error).
 * - Nodal vectors are C-ordered with x slowest: u[(i*n + j)*n + k].  The
 *   first Kronecker factor acts on x.
 * - Argument errors (null pointers, n outside [2,32], dim not 2 or 3, rank
 *   not supported) return KP_ERR_ARG and write nothing.  HIP runtime errors
 *   return KP_ERR_HIP.  Per-element numerical trouble is reported in
 *   elem_status (bit flags KP_ELEM_*) and is not an error of the call.
 *   No C++ exception crosses this interface.
 */
#ifndef KP_H
#define KP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct kp_ctx_s* kp_ctx;

typedef enum {
    KP_OK = 0,
    KP_ERR_ARG = 1,
    KP_ERR_ALLOC = 2,
    KP_ERR_HIP = 3,
    KP_ERR_NUMERIC = 4,
    KP_ERR_NOCONV = 5,
    KP_ERR_UNSUPPORTED = 6
} kp_status;

/* Arithmetic of the apply.  KP_BF16: bf16 operands, FP32 accumulation.
 * KP_BF16X3: every operand split as hi + lo bf16 numbers and each product
 * formed from the three terms hi*hi + hi*lo + lo*hi with FP32 accumulation
 * (about 16 significant bits at the bf16 matrix-core rate). */
typedef enum { KP_FP64 = 0, KP_FP32 = 1, KP_BF16 = 2, KP_BF16X3 = 3 } kp_prec;

/* setup modes for kp_setup */
typedef enum { KP_SETUP_SVD = 0, KP_SETUP_LEARNED = 1, KP_SETUP_LEARNED_WARM = 2 } kp_setup_mode;

/* preconditioner kinds for kp_fgmres */
typedef enum { KP_PC_NONE = 0, KP_PC_KSVD = 1, KP_PC_BJ = 2 } kp_pc_kind;

/* per-element status bits */
#define KP_ELEM_OK 0
#define KP_ELEM_LANCZOS_NOCONV 1    /* Lanczos hit its step limit; best Ritz triplets used */
#define KP_ELEM_SINGULAR_FACTOR 2   /* a factor to invert had a zero pivot */
#define KP_ELEM_SCHUR_NOCONV 4      /* Francis QR did not converge */
#define KP_ELEM_NONFINITE 8         /* NaN/Inf in the element's data or results */
#define KP_ELEM_LEARNED_REJECTED 16 /* learned factors failed the acceptance test */
#define KP_ELEM_LEARNED_WARM 32     /* the factors come from a Lanczos run started at the prediction */

#define KP_REC_LEN 16

/*
 * A batch of elements of one dimension and one degree.
 *   params : [E][16] element records (always required).  Record layout:
 *            [0..2] beta_x, beta_y, beta_z (element velocity a = -beta),
 *            [3] nu, [4] alpha, [5] phi, [6] tau, [7] face flag,
 *            [8..13] normal velocity u_f of the upwind flux on the faces
 *            x-, x+, y-, y+, z-, z+ (outward normal, u_f > 0 outflow),
 *            [14..15] zero.
 *            The block of element k is (Sec. 3.4, Table 1, eq. adv-kron, with
 *            collocated Gauss-Legendre quadrature on [0,1]^d):
 *              diag(w (x) w [(x) w] * c) + tau * sum_axes (beta S + nu K) on
 *              that axis (x) W on the others, c = 1 + alpha sin(pi x y [z] + phi),
 *            plus, if face != 0, the outflow self-term tau*u_f * l l^T on the
 *            face's axis (l = l(0) low face, l(1) high face) (x) W on the others
 *            for every face with u_f > 0.
 *   blocks : [E][n^d][n^d] explicit blocks, row-major, or NULL.  When NULL the
 *            setup and the operator are matrix-free from params.
 *   nbr    : [E][2*dim] face neighbours (low, high per axis), or NULL.  Used
 *            only by kp_operator_apply and kp_fgmres for the upwind coupling:
 *            on a face with u_f < 0 the element receives
 *            tau*u_f (l_f l_opp^T (x) W ...) applied to the neighbour's values.
 */
typedef struct {
    int64_t num_elems;
    int32_t dim;
    int32_t n;
    const double* params;
    const double* blocks;
    const int32_t* nbr;
} kp_batch;

/* Context bound to one device and one HIP stream (hipStream_t passed as void*;
 * NULL means the default stream). */
kp_status kp_create(kp_ctx* ctx, int device, void* stream);
kp_status kp_destroy(kp_ctx ctx);
kp_status kp_set_stream(kp_ctx ctx, void* stream);

/* Context options (kp_set_option):
 *   KP_OPT_FGMRES_GRAPHS (default 0): run every restart cycle of kp_fgmres /
 *     kp_mixed_fgmres / kp_fgmres_sys as one HIP graph (per Arnoldi step the
 *     preconditioner, the operator, both Gram-Schmidt passes, the norm and the
 *     normalisation of the next basis vector on the device; then one copy of
 *     the cycle's projections into pinned host memory), captured once per
 *     solve on a private stream and replayed every cycle, with one
 *     synchronisation per cycle instead of one per step.  The host applies the
 *     Givens rotations to the cycle's columns afterwards and stops at the same
 *     column as without graphs, so iterations and solution are the same; the
 *     last cycle's steps after that column run without effect.  A cycle that
 *     cannot be captured runs without graphs.
 *   KP_OPT_APPLY_MFMA16 (default 1): the matrix-core apply for n = 16; 0
 *     selects the generic per-element kernel.
 *   KP_OPT_FGMRES_Z32 (default 1): kp_fgmres keeps the preconditioned basis
 *     Z in FP32 when the preconditioner is the rank-2 KSVD apply in FP32,
 *     BF16 or split BF16 (kp_apply_z32); its outputs are FP32 numbers, so
 *     the solve is the same as with an FP64 basis, with half the basis
 *     bytes; 0 keeps Z in FP64.
 *   KP_OPT_OPERATOR_COLS (default 1): kp_operator_apply and kp_fgmres apply
 *     the matrix-free operator of 3D batches with n <= 16 with one thread per
 *     column of each element (the element structure formed first); the
 *     entries are formed from the same terms in the same order as by the
 *     one-entry-per-thread kernel (equal to rounding); 0 selects that
 *     kernel.
 *   KP_OPT_LEARNED_GUARD (default 10000): the spectral guard of the learned
 *     setup (kp_setup mode KP_SETUP_LEARNED) in millionths: a prediction is
 *     used only if its estimate of ||P_svd^{-1} P_pred - I||_2 is at most
 *     value * 1e-6 (default 0.01).  Values in [0, 1000000].  At 3D p = 15 a
 *     guard of 0.1 lets through predictions that cost FGMRES(30) 32 more
 *     iterations (258 against 226); 0.01 keeps the count.
 *   KP_OPT_SPLIT_AXIS (default 0): 3D only.  0: the rank-1 stage of the
 *     two-stage KSVD splits the x axis, as the paper does (Sec. 4.3.1).  1:
 *     kp_setup forms the two-stage KSVD with the split on each of x, y and z
 *     and keeps, per element, the one whose rank-1 stage keeps the most of
 *     ||A||_F (the largest stage-1 sigma_1; ties to x); kp_get_axes reports
 *     the choice.  Factors are then in the element's relabelled axis order
 *     (y,x,z for y; z,x,y for z), and kp_apply / kp_apply_z32 / kp_fgmres on
 *     the same context load and store each element's tensor in that order.
 *     Records only (the record's mass coefficient is symmetric in the axes,
 *     so the relabelled block is that of the record with its per-axis data
 *     permuted); explicit 3D blocks, the learned modes and kp_setup_noalloc
 *     return KP_ERR_UNSUPPORTED.  A preconditioner formed with the option on
 *     must be applied with it on.  Three times the Lanczos work of the setup.
 *   KP_OPT_APPLY_SMALL3 (default 1): the 3D apply for n <= 8 runs one wave
 *     per (element, right-hand side) with the tensor held as register fibres
 *     (the arithmetic of the generic apply); 0 selects the generic
 *     per-element kernel. */
typedef enum {
    KP_OPT_FGMRES_GRAPHS = 1,
    KP_OPT_APPLY_MFMA16 = 2,
    KP_OPT_FGMRES_Z32 = 3,
    KP_OPT_OPERATOR_COLS = 4,
    KP_OPT_LEARNED_GUARD = 5,
    KP_OPT_SPLIT_AXIS = 6,
    KP_OPT_APPLY_SMALL3 = 7
} kp_option;
kp_status kp_set_option(kp_ctx ctx, int32_t option, int64_t value);
const char* kp_status_string(kp_status s);

/* Bytes of the opaque preconditioner buffer for a batch and rank.
 * rank: 2D: 1, 2 or 3; 3D: 2 (the two-stage form of Sec. 4.3.1).  Returns 0
 * for an unsupported combination.  The buffer holds, per element, the
 * singular values, the Kronecker factors in FP64 and the apply tables in
 * FP64, FP32 and BF16; kp_get_factors reads the factors back. */
size_t kp_precond_bytes(int32_t dim, int32_t n, int32_t rank, int64_t num_elems);

/* Materialise the explicit blocks of a batch from its records
 * (out: [E][n^d][n^d] row-major FP64). */
kp_status kp_build_blocks(kp_ctx ctx, const kp_batch* b, double* out);

/* Form the preconditioner (Alg. 5 in 2D, Alg. 7 in 3D).
 * Lanczos (Alg. 2, full reorthogonalisation) on the rearranged block R(A_k)
 * through matrix-free products (explicit blocks when b->blocks != NULL,
 * otherwise the sum-factorised products of Sec. 4.2.1 / 4.3.2 from the
 * records), factors vec(A_j) = sqrt(sigma_j) u_j, vec(B_j) = sqrt(sigma_j) v_j,
 * then LU inverses and real Schur forms in FP64 and the apply tables.
 * mode KP_SETUP_LEARNED (rank 2, records only, a model for this dim and n
 * attached with kp_set_model; 3D n <= 16): the network predicts every
 * element's factors; the SVD setup runs as judge and fallback, its Lanczos
 * started from the predicted vec(A1) (in 3D the second stage from vec(B1)),
 * and cold where that does not converge; then kp_learned_judge with factor
 * 1.1 and the guard of KP_OPT_LEARNED_GUARD decides per element.  Accepted elements keep the
 * predicted factors (status 0); rejected ones keep the SVD's (status
 * KP_ELEM_LEARNED_REJECTED, plus KP_ELEM_LEARNED_WARM when the warm-started
 * Lanczos converged).  sigma holds the SVD's singular values either way.
 * The judge needs the SVD, so this mode costs more than KP_SETUP_SVD.
 * mode KP_SETUP_LEARNED_WARM: every element runs the Lanczos setup started
 * from the prediction, status KP_ELEM_LEARNED_WARM, with the cold fallback
 * (status 0); the factors are the SVD's to the Lanczos tolerance.
 * precond: kp_precond_bytes bytes.  elem_status: [E] int32, or NULL. */
kp_status kp_setup(kp_ctx ctx, const kp_batch* b, int32_t rank, int32_t mode,
                   void* precond, int32_t* elem_status);

/* kp_setup without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  SVD mode only; same arguments, outputs and per-element status
 * as kp_setup(ctx, b, rank, KP_SETUP_SVD, precond, elem_status), and the same
 * preconditioner bytes.  The Lanczos workspace lives in a static device array
 * of 128 MiB per device (held until the process ends); the 1D tables were
 * built by kp_create.  Batches whose per-element workspace needs more than a
 * quarter of that array (four slots) return KP_ERR_UNSUPPORTED; a batch with
 * fewer slots than kp_setup would use runs with fewer workgroups.  Every call
 * on one device shares the array: calls that overlap in time on one device
 * (two streams, two contexts, two threads) race and must be serialised by the
 * caller.  Nothing in the array needs to start at zero.  KP_ERR_HIP if the
 * array's device address could not be resolved at kp_create. */
kp_status kp_setup_noalloc(kp_ctx ctx, const kp_batch* b, int32_t rank, void* precond,
                           int32_t* elem_status);

/* Judge predicted rank-2 factors against the SVD's (the learned setup's
 * acceptance test; not in the paper, which always takes the SVD, Sec. 4.1).
 * pred_factors: [E][nf][n][n] FP64 (3D: A1,B1,C1,B2,C2; 2D: A1,B1,A2,B2);
 * precond: a KP_SETUP_SVD preconditioner of the same batch (its factors and
 * FP64 apply tables are the judge).  Per element, with A the record's block:
 *   out[e][0] = ||A - P_pred||_F, out[e][1] = ||A - P_svd||_F (both in
 *   closed form from the record), out[e][2] = ||A||_F,
 *   out[e][3] = gamma, a three-step power estimate of
 *   ||P_svd^{-1} P_pred - I||_2 from the normalised ones vector (a lower
 *   bound of that norm);
 *   accept[e] = 1 iff out0 <= factor * out1, out0 < out2 and gamma <= guard.
 * Records only (b->blocks NULL), rank 2, 3D n <= 16.  out or accept may be
 * NULL (not both). */
kp_status kp_learned_judge(kp_ctx ctx, const kp_batch* b, int32_t rank, const double* pred_factors,
                           const void* precond, double factor, double guard, double* out,
                           int32_t* accept);

/*
 * A batch of general elements of one dimension and one degree, given by
 * their coefficients at mu >= n Gauss-Legendre points per axis of [0,1]
 * (non-collocated quadrature, Sec. 3.4.1): the data a DG code's linearisation
 * hands over on curved elements.  All device pointers, C order, x slowest:
 *   c  [E][mu^d]      mass coefficient (|det J| times the pointwise mass factor)
 *   a  [E][d][mu^d]   flux-Jacobian component dF_i/du
 *   nu [E][mu^d]      second-order coefficient
 *   g  [E][2d][mu^(d-1)]  upwind face coefficient on face 2*axis + side, at the
 *                         face's own points (the other axes in order)
 * With the Lagrange basis phi on the n Gauss-Legendre nodes and weights w,
 * element k's block (rows test, columns trial functions) is
 *   sum_q w_q c_q phi_I phi_K - tau sum_i sum_q w_q a_i(q) (d_i phi_I) phi_K
 *   + tau sum_i sum_q w_q nu_q (d_i phi_I)(d_i phi_K)
 *   + tau sum_f sum_{q on f} w_q g_f(q) phi_I phi_K   (eq. jac-entries).
 */
typedef struct {
    int64_t num_elems;
    int32_t dim, n, mu, pad;
    double tau;
    const double* c;
    const double* a;
    const double* nu;
    const double* g;
} kp_quad_batch;

/* Form the rank-2 preconditioner (2D: rank 2; 3D: the two-stage form) of a
 * batch of general elements (Sec. 4.1, Sec. 4.3.1, with the products of
 * Sec. 4.2.1 / 4.3.2).  Lanczos on R(A) R(A)^T in its Gram form: the
 * rearranged block of every term is X_p^T F Y with X_p[alpha,(a,c)] =
 * L_p[alpha,a] R_p[alpha,c], so R R^T x needs the coefficient tensors and the
 * small Grams X_p X_q^T only (O(mu^3) per step in 3D; no vector of length
 * n^4); the stage-1 right factor D1 stays in that factored form for stage 2.
 * precond: kp_precond_bytes(dim, n, 2, E) bytes, used by kp_apply /
 * kp_fgmres with a kp_batch of the same E, dim, n (params may be NULL there).
 * 2 <= n <= mu <= 32.  elem_status as for kp_setup. */
kp_status kp_setup_quad(kp_ctx ctx, const kp_quad_batch* q, void* precond, int32_t* elem_status);

/* Explicit diagonal blocks of a 2D system of nc coupled components (Sec. 5.3,
 * the Euler and Navier-Stokes experiments: blocks of size nc (p+1)^2).  Nodal
 * vectors are ordered (component, x, y), component slowest, so the first
 * Kronecker factor acts on the pair (component, x):
 *   A_k ~ A1 (x) B1 + A2 (x) B2,  A_j: m x m with m = nc n,  B_j: n x n.
 * blocks: device, [E][m n][m n] FP64 row-major.  1 <= nc, 2 <= n,
 * nc n <= 32.  nc = 1 is the scalar 2D block. */
typedef struct {
    int64_t num_elems;
    int32_t nc, n;
    const double* blocks;
} kp_sys_batch;

/* Bytes of the preconditioner buffer of a systems batch (0 if nc, n are out
 * of range).  It holds, per element, the factors [A1 m^2, B1 n^2, A2 m^2,
 * B2 n^2] and sigma[4] in FP64, and the apply tables in FP64 and FP32. */
size_t kp_sys_precond_bytes(int32_t nc, int32_t n, int64_t num_elems);

/* Form the rank-2 preconditioner of a systems batch (Sec. 4.1 with m1 = n1 =
 * nc n, m2 = n2 = n; Alg. 5): Lanczos (Alg. 2) on the n^2 x n^2 Gram
 * R(A)^T R(A), left vectors u_j = R(A) v_j / sigma_j, each pair signed so that
 * the largest-magnitude entry of A_j is positive; then C1 = A2^-1 A1,
 * C2 = B1^-1 B2, their real Schur forms, and the Sylvester sweep's column
 * inverses (TA + t_jj I)^-1 (for a 2 x 2 block of TB, ((TA + pI)^2 - qs I)^-1)
 * in FP64, with an FP32 copy.  elem_status: [E] int32 device, or NULL; bits
 * as for kp_setup (1 Lanczos not converged, 2 singular factor, 4 Schur not
 * converged, 8 non-finite tables).  The setup workspace (about
 * (n^4 + 6 m^2 + 64 n^2) doubles per workgroup, at most 2048 workgroups) is
 * allocated on the context and kept. */
kp_status kp_setup_sys(kp_ctx ctx, const kp_sys_batch* b, void* precond, int32_t* elem_status);

/* z = P^{-1} r per element (Alg. 6 with an m x m first factor): for X the
 * element's vector as an m x n matrix (rows (component, x), columns y),
 * X -> QA^T A2^-1 X B1^-T QB, the quasi-triangular Sylvester sweep
 * TA S + S TB^T = F over the columns of TB from the last, then QA S QB^T.
 * r, z: device, [E][nrhs][m n] FP64.  prec KP_FP64 or KP_FP32 (tables and
 * arithmetic); other precisions return KP_ERR_UNSUPPORTED.  b->blocks may be
 * NULL. */
kp_status kp_apply_sys(kp_ctx ctx, const kp_sys_batch* b, const void* precond, int32_t prec, int32_t nrhs,
                       const double* r, double* z);

/* Copy factors ([E][2 m^2 + 2 n^2] in the order above) and singular values
 * ([E][4]: sigma_1, sigma_2, 0, 0) out of a systems preconditioner (device
 * pointers; either may be NULL). */
kp_status kp_get_factors_sys(kp_ctx ctx, const kp_sys_batch* b, const void* precond, double* factors,
                             double* sigma);

/* Element records of a systems batch, for kp_build_sys_blocks:
 * [E][6 nc^2 + 5] FP64 = Jx, Jy, Jx+, Jy+, Jx-, Jy- (nc x nc flux Jacobians,
 * row-major; J+ = (J)^+ the outflow part of the upwind flux through the high
 * face of that axis, J- = (-J)^+ through the low face), nu, alpha, phi, tau,
 * face flag.  Element k's block (Sec. 3.4, eq. adv-kron with the advection
 * velocity replaced by the Jacobians; collocated Gauss-Legendre quadrature):
 *   I (x) diag(w (x) w * c) + tau [-Jx (x) S (x) W - Jy (x) W (x) S
 *     + nu I (x) (K (x) W + W (x) K)]
 *   + tau [Jx+ (x) l1 l1^T (x) W + Jx- (x) l0 l0^T (x) W
 *     + Jy+ (x) W (x) l1 l1^T + Jy- (x) W (x) l0 l0^T]   (if face != 0),
 * c = 1 + alpha sin(pi x y + phi).  blocks: [E][nc n^2][nc n^2] FP64. */
kp_status kp_build_sys_blocks(kp_ctx ctx, int64_t num_elems, int32_t nc, int32_t n, const double* recs,
                              double* blocks);

/* y = blockdiag(A_k) x for a systems batch (no coupling between elements).
 * x, y: [E][nc n^2]. */
kp_status kp_sys_operator_apply(kp_ctx ctx, const kp_sys_batch* b, const double* x, double* y);

/* Exact block Jacobi of a systems batch: LU with partial pivoting of every
 * (nc n^2) x (nc n^2) block (the blocked kernel of kp_blockjacobi_exact).
 * lu: [E][N][N], piv: [E][N] (N = nc n^2); elem_status as there. */
kp_status kp_sys_blockjacobi_exact(kp_ctx ctx, const kp_sys_batch* b, double* lu, int32_t* piv,
                                   int32_t* elem_status);

/* FGMRES(restart) on blockdiag(A_k) x = rhs from x = 0, as kp_fgmres:
 * pc_kind KP_PC_KSVD (pc_data = kp_setup_sys buffer, applied in pc_prec
 * KP_FP64 or KP_FP32), KP_PC_BJ (pc_data = lu, pc_aux = piv from
 * kp_sys_blockjacobi_exact) or KP_PC_NONE.  Same stopping rule, workspace
 * and synchronisation as kp_fgmres; iters_h, relres_h host scalars. */
kp_status kp_fgmres_sys(kp_ctx ctx, const kp_sys_batch* b, int32_t pc_kind, const void* pc_data,
                        const void* pc_aux, int32_t pc_prec, const double* rhs, double* x, int32_t restart,
                        double rtol, int32_t maxit, int32_t* iters_h, double* relres_h);

/* Build only the apply tables from given Kronecker factors
 * (factors: [E][nf][n][n] FP64, 2D rank r: A1,B1,A2,B2,...; 3D: A1,B1,C1,B2,C2). */
kp_status kp_setup_from_factors(kp_ctx ctx, const kp_batch* b, int32_t rank,
                                const double* factors, void* precond, int32_t* elem_status);

/* Copy the factors ([E][nf][n][n]) and singular values ([E][4]: 2D sigma_1..r;
 * 3D sigma_1 of stage 1, then sigma_1, sigma_2 of stage 2) out of a
 * preconditioner buffer.  Either output may be NULL. */
kp_status kp_get_factors(kp_ctx ctx, const kp_batch* b, int32_t rank, const void* precond,
                         double* factors, double* sigma);

/* Copy the 3D elements' split axes ([E] int8: 0 = x, 1 = y, 2 = z) out of a
 * preconditioner buffer (all 0 unless formed under KP_OPT_SPLIT_AXIS). */
kp_status kp_get_axes(kp_ctx ctx, const kp_batch* b, int32_t rank, const void* precond, int8_t* axes);

/* z = P^{-1} r per element (Alg. 6 in 2D, Alg. 8 in 3D) for nrhs
 * right-hand sides.  r, z: [E][nrhs][n^d] FP64.  prec selects the arithmetic
 * of the contractions and the Sylvester solve (FP64, FP32, or BF16 operands
 * with FP32 accumulation).
 * 2D rank 3: the paper gives no direct inverse for more than two Kronecker
 * terms (Sec. 4.2), so P = A1(x)B1 + A2(x)B2 + A3(x)B3 is solved per element by
 * flexible GMRES (restart 8, at most 200 iterations, FP64 Arnoldi and
 * Kronecker products) preconditioned by the rank-2 apply of the first two
 * terms in precision prec, to a relative residual of 1e-13 (FP64), 1e-10
 * (FP32), 1e-6 (BF16) or 1e-9 (split BF16).  An element that misses its
 * target within the limit returns its last iterate. */
kp_status kp_apply(kp_ctx ctx, const kp_batch* b, int32_t rank, const void* precond,
                   int32_t prec, int32_t nrhs, const double* r, double* z);

/* kp_apply with z stored in FP32: z [E][nrhs][n^d] float.  For rank 2 and
 * prec FP32, BF16 or split BF16, whose apply ends in FP32 arithmetic: every
 * stored value equals the one kp_apply writes as FP64 (the FP32 number it
 * holds), with half the output bytes.  Rank 3 and prec FP64 return
 * KP_ERR_UNSUPPORTED (their outputs are FP64 numbers); other arguments as in
 * kp_apply. */
kp_status kp_apply_z32(kp_ctx ctx, const kp_batch* b, int32_t rank, const void* precond,
                       int32_t prec, int32_t nrhs, const double* r, float* z);

/* Exact block Jacobi (the paper's comparator, Sec. 5).  Factor every explicit
 * block b->blocks by LU with partial pivoting: lu [E][N][N] row-major per
 * element (entry (i,j) at i*N + j; unit lower triangle below the diagonal, U
 * on and above), piv [E][N] (row swapped with row k at step k), N = n^d <=
 * 4096.  lu may be b->blocks itself (factored in place: 64 GiB instead of 128
 * for 32768 blocks of 512 x 512).  Blocked right-looking LU, the trailing
 * updates on the FP64 matrix cores.  A zero pivot sets
 * KP_ELEM_SINGULAR_FACTOR in elem_status (may be NULL).  Then z = A_k^{-1} r
 * for nrhs right-hand sides ([E][nrhs][N]). */
kp_status kp_blockjacobi_exact(kp_ctx ctx, const kp_batch* b, double* lu, int32_t* piv,
                               int32_t* elem_status);
kp_status kp_blockjacobi_solve(kp_ctx ctx, const kp_batch* b, const double* lu,
                               const int32_t* piv, int32_t nrhs, const double* r, double* z);

/* y = G x for the global operator: diagonal blocks (explicit or
 * matrix-free) plus the upwind inflow coupling through nbr. x, y: [E][n^d].
 * Matrix-free 3D batches with n <= 16 (KP_OPT_OPERATOR_COLS) first form the
 * element structure into ctx workspace ((n^3 + 3 n^2) doubles per element). */
kp_status kp_operator_apply(kp_ctx ctx, const kp_batch* b, const double* x, double* y);

/* FGMRES(restart) on G x = rhs from x = 0 with flexible right
 * preconditioning (Sec. 5: restarted preconditioned GMRES): pc_kind KP_PC_KSVD
 * (pc_data = kp_setup buffer of this rank, applied in pc_prec), KP_PC_BJ
 * (pc_data = lu, pc_aux = piv from kp_blockjacobi_exact) or KP_PC_NONE.
 * Classical Gram-Schmidt applied twice, Givens rotations on the host.  Stops
 * when the residual estimate is <= rtol*||rhs|| and the true residual
 * recomputed at the restart confirms it, or after maxit Arnoldi steps (then
 * KP_ERR_NOCONV; x holds the last iterate).  Synchronises once per Arnoldi
 * step (once per cycle under KP_OPT_FGMRES_GRAPHS).  iters_h, relres_h: host
 * scalars (final true relative residual); hist_h: host array of hist_len
 * per-step relative residual estimates, or NULL.  Workspace:
 * (2*restart + 3) * E * n^d doubles (the basis Z in FP32 under
 * KP_OPT_FGMRES_Z32: restart/2 fewer), owned by ctx. */
kp_status kp_fgmres(kp_ctx ctx, const kp_batch* b, int32_t pc_kind, int32_t rank,
                    const void* pc_data, const void* pc_aux, int32_t pc_prec, const double* rhs,
                    double* x, int32_t restart, double rtol, int32_t maxit, int32_t* iters_h,
                    double* relres_h, double* hist_h, int32_t hist_len);

/* ------------------------------------------------------ mixed batches
 * Elements of different dimension and degree in one batch (records
 * [E][16] as for kp_batch, block-diagonal: no face coupling).  Vectors are
 * packed in element order: element e holds its n_e^d_e values after those of
 * the elements before it.  A plan holds the layout and the per-element
 * descriptors that let one persistent launch serve the whole batch; the
 * setup, the apply and the block-diagonal operator each take one launch
 * (the setup also runs the three table kernels and the precision copies).
 * Rank 2 (2D) and the two-stage rank-2 form (3D), SVD setup. */
typedef struct kp_mixed_plan_s* kp_mixed_plan;

/* dim_n_h: host [E][2] = (dim, n) per element, dim 2 or 3, 2 <= n <= 32.
 * Allocates the plan's device descriptors (owned by the plan). */
kp_status kp_mixed_plan_create(kp_ctx ctx, int64_t num_elems, const int32_t* dim_n_h, kp_mixed_plan* plan);
kp_status kp_mixed_plan_destroy(kp_mixed_plan plan);

/* Packed vector length (sum of n_e^d_e) and preconditioner bytes. */
kp_status kp_mixed_plan_info(kp_mixed_plan plan, int64_t* vec_len_h, size_t* precond_bytes_h);

/* Setup of every element (Alg. 5 / Alg. 7 with its own n); elem_status [E] or NULL.
 * Ordered on ctx's stream as a whole: the table kernels of the (dim, n)
 * classes run concurrently on three side streams that the plan owns (created
 * at the first setup, default priority, destroyed with the plan), forked from
 * and joined back to ctx's stream with events.  Calls on one plan must not
 * overlap. */
kp_status kp_mixed_setup(kp_ctx ctx, kp_mixed_plan plan, const double* params, void* precond,
                         int32_t* elem_status);

/* Factors (packed: 4 n_e^2 doubles per 2D element, 5 n_e^2 per 3D element, in
 * element order) and sigma [E][4]; either may be NULL. */
kp_status kp_mixed_get_factors(kp_ctx ctx, kp_mixed_plan plan, const void* precond, double* factors,
                               double* sigma);

/* z = P^{-1} r for every element in one launch (r, z packed). */
kp_status kp_mixed_apply(kp_ctx ctx, kp_mixed_plan plan, const void* precond, int32_t prec,
                         const double* r, double* z);

/* Autotune the apply launch: for every (dim, n) in the batch, time its
 * elements applied by a whole workgroup each and by one wave each (four per
 * workgroup), keep the faster, and rebuild the plan's work list.  The wave
 * mode is tried only where four elements' three FP64 buffers fit in 150 KiB
 * of LDS (every 2D n up to 40, 3D n up to 11), so the chosen work list serves
 * every precision.  r and z
 * are used as scratch (z is overwritten).  modes_h (or NULL): triples
 * (dim, n, mode 0 workgroup / 1 wave), -1 after the last.  Synchronises. */
kp_status kp_mixed_autotune(kp_ctx ctx, kp_mixed_plan plan, const void* precond, int32_t prec,
                            const double* r, double* z, int32_t* modes_h, int32_t modes_len);

/* y = blockdiag(A_e) x from the records (packed vectors). */
kp_status kp_mixed_operator_apply(kp_ctx ctx, kp_mixed_plan plan, const double* params, const double* x,
                                  double* y);

/* FGMRES(restart) on the block-diagonal system of the batch, as kp_fgmres;
 * pc_kind KP_PC_KSVD (precond from kp_mixed_setup, applied in pc_prec) or
 * KP_PC_NONE. */
kp_status kp_mixed_fgmres(kp_ctx ctx, kp_mixed_plan plan, const double* params, int32_t pc_kind,
                          const void* precond, int32_t pc_prec, const double* rhs, double* x,
                          int32_t restart, double rtol, int32_t maxit, int32_t* iters_h, double* relres_h,
                          double* hist_h, int32_t hist_len);

/* ------------------------------------------------------ learned setup
 * Not part of the paper, whose SVD setup (Sec. 4.1) stays the arbiter.  A small
 * MLP maps 12 features of an element record to its Kronecker factors:
 *   features: beta_x, beta_y, beta_z (0 in 2D), log10 nu, tau, alpha, sin phi,
 *     cos phi, and c = 1 + alpha sin(pi x y [z] + phi) at the reference
 *     points (1/4,1/4,1/4), (3/4,1/4,3/4), (1/4,3/4,3/4), (3/4,3/4,1/4)
 *     (2D: the same (x, y));
 *   xn = (features - x_mean) / x_std, h1 = silu(W1 xn + b1),
 *   h2 = silu(W2 h1 + b2), y = W3 h2 + b3 (W1: H x 12, W2: H x H, W3: O x H,
 *   row-major FP32; silu(z) = z / (1 + e^-z));
 *   factors = y times a scale per factor block, O = 5 n^2 in 3D
 *   (A1,B1,C1,B2,C2), 4 n^2 in 2D rank 2 (A1,B1,A2,B2).
 * The model is one opaque device buffer of kp_mlp_bytes bytes holding a
 * header, the parameters (W1,b1,W2,b2,W3,b3 in that order, P floats), the
 * Adam moments and the normalisation.  prec for the network: KP_FP32 (FP32
 * matrix-core GEMMs) or KP_BF16 (bf16 operands, FP32 accumulation).
 * Training loss: mean squared error of the scaled outputs, each sample
 * compared with the sign pattern of its target closest to the prediction
 * among the sign changes that leave P unchanged (3D: A1 -> s0 A1,
 * B_j -> s_j B_j, C_j -> s0 s_j C_j; 2D: (A_j, B_j) -> s_j (A_j, B_j)). */

/* Bytes of a model for (dim, n) and H hidden units; 0 if unsupported. */
size_t kp_mlp_bytes(int32_t dim, int32_t n, int32_t hidden);

/* Write the header, copy params (P FP32 values, device) or zeros when NULL,
 * clear the optimiser state, set x_mean = 0, x_std = 1, scales = 1.
 * Synchronises. */
kp_status kp_mlp_init(kp_ctx ctx, void* model, int32_t dim, int32_t n, int32_t hidden,
                      const float* params);

/* Copy parameters (P), x_mean (12), x_std (12), block scales (5 or 4) out of
 * a model; any output may be NULL. */
kp_status kp_mlp_get(kp_ctx ctx, const void* model, float* params, float* x_mean, float* x_std,
                     float* yscale);

/* Overwrite the normalisation of a model (any argument may be NULL). */
kp_status kp_mlp_set_norm(kp_ctx ctx, void* model, const float* x_mean, const float* x_std,
                          const float* yscale);

/* y = network(xn) for rows normalised inputs xn [rows][12]; y: [rows][O]
 * scaled outputs. */
kp_status kp_mlp_forward(kp_ctx ctx, const void* model, int32_t prec, int64_t rows, const float* xn,
                         float* y);

/* Loss of rows samples (xn [rows][12], scaled targets t [rows][O]) and its
 * gradient with respect to the parameters (grad: P floats, loss: 1 float,
 * both device). */
kp_status kp_mlp_loss_grad(kp_ctx ctx, const void* model, int32_t prec, int64_t rows, const float* xn,
                           const float* t, float* grad, float* loss);

/* Train on a batch of elements and their SVD factors (factors [E][O] FP64,
 * the kp_get_factors layout): features and their mean / standard deviation
 * and the per-block RMS scales of the targets are computed and stored in the
 * model, then epochs passes of Adam (beta1 0.9, beta2 0.999, eps 1e-8,
 * learning rate lr) over minibatches of `batch` elements in an order drawn
 * by a splitmix64 / Fisher-Yates shuffle from seed.  loss_hist_h: host array
 * of epochs mean minibatch losses, or NULL.  Synchronises once per epoch. */
kp_status kp_mlp_train(kp_ctx ctx, void* model, const kp_batch* b, const double* factors,
                       int32_t epochs, int32_t batch, float lr, uint64_t seed, int32_t prec,
                       float* loss_hist_h);

/* Predicted factors of a batch ([E][O] FP64) from its records. */
kp_status kp_mlp_predict(kp_ctx ctx, const void* model, const kp_batch* b, int32_t prec,
                         double* factors);

/* Attach a model to the context for kp_setup(mode = KP_SETUP_LEARNED); NULL
 * detaches.  The model must stay alive and unchanged while attached. */
kp_status kp_set_model(kp_ctx ctx, const void* model);

#ifdef __cplusplus
}
#endif

#endif /* KP_H */
