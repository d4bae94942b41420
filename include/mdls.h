/*
 * mdls.h -- multiple-double least squares on AMD MI355X (gfx950): the C ABI.
 *
 * Solves min || b - A x ||_2 for a full-column-rank A (m x n, m >= n) in double double,
 * quad double or octo double arithmetic: numbers are unevaluated sums of P = 2, 4 or 8
 * doubles (paper Section 1.1).  The method is the paper's: Householder QR of A (Section 3,
 * Algorithm 2, with the sign choice of Golub and Van Loan Algorithm 5.1.1), the product
 * Q^T b, and the tiled back substitution of R x = Q^T b (Section 2, Algorithm 1: invert the
 * diagonal tiles, then alternate x_i = U_i^{-1} b_i with the updates b_j -= A_{j,i} x_i).
 *
 * Storage (the paper's staging, end of Section 2): a matrix of multiple doubles is P planes
 * of doubles, most significant limb first.  Plane k starts ld * cols doubles after plane
 * k - 1 and is column-major with leading dimension ld >= rows.  A vector of length L is P
 * planes of L doubles.  Every pointer below is a DEVICE pointer unless it says HOST.  The
 * caller owns every buffer; the library never allocates device memory or frees, and
 * synchronises only in the set-up and tuning calls that say so (mdls_init, mdls_finalize,
 * mdls_batch_plan, mdls_batch_autotune).  Work is enqueued on the caller's stream.  After
 * mdls_init on the calling host thread, the QR also forks part of each trailing update onto a
 * side stream that mdls_init created for that thread and device (default priority), and joins
 * it back with events before returning; the caller's stream still orders everything, and a
 * call can be captured into a HIP graph.  Without mdls_init every kernel runs on the caller's
 * stream (same results, bit for bit).  No solve call creates a stream or an event.
 *
 * Errors: a call returns 0 on success; -i when argument i (1-based) is invalid, checked on
 * the host before anything is enqueued (LAPACK convention); MDLS_EHIP when a launch fails;
 * MDLS_EUNSUPPORTED for valid arguments the library does not handle (too many rows for the
 * panel kernel, or a device with too few compute units for its workgroups).
 * Numerical status is written asynchronously to the device int *d_info where a call has
 * one: 0 = success, k > 0 = R(k,k) is exactly zero (1-based), x then unspecified; -1 = a
 * grid barrier of the factorisation gave up waiting (see below), the results are unspecified.
 * NaN and Inf in the input propagate to the output unchecked (d_info stays 0 unless R(k,k) is
 * exactly zero).  No call throws.
 *
 * Co-residency: a Householder panel of more than one workgroup synchronises its workgroups
 * once per column with a grid barrier, so all of them must be resident at once.  The library
 * checks that the panel's workgroups fit the device (occupancy x compute units) and otherwise
 * returns MDLS_EUNSUPPORTED; the concurrent trailing update never waits, so it cannot block
 * them.  Work of other processes or streams that holds compute units for longer than the
 * barrier's spin limit (about 0.1 s by default) can still make a barrier give up: it then
 * lets its workgroup continue, every kernel exits normally, and *d_info reports -1.
 *
 * Threading: calls on distinct streams with distinct buffers and workspaces may run
 * concurrently.  One workspace must not be used by two calls in flight at once.
 */
#ifndef MDLS_H
#define MDLS_H

#include <stddef.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* precision = number of limbs P.  MDLS_F64 (one limb) exists for tests only. */
typedef enum { MDLS_F64 = 1, MDLS_DD = 2, MDLS_QD = 4, MDLS_OD = 8 } mdls_prec;

#define MDLS_EHIP (-100)        /* a kernel launch failed */
#define MDLS_EUNSUPPORTED (-101) /* valid arguments outside what the library handles */
#define MDLS_ESCRATCH (-102)     /* mdls_solve_noalloc: the workspace would exceed its static scratch */

/*
 * Set-up of the calling host thread on the current device: creates the look-ahead side stream
 * and its events, and queries the panel kernels' occupancy.  Call it before the first solve
 * (and before any graph capture) on each thread that wants the concurrent trailing update;
 * repeated calls do nothing.  mdls_finalize waits for the side stream and destroys it (the
 * thread's later calls then run on the caller's stream alone).  Both return 0 or MDLS_EHIP
 * (MDLS_EUNSUPPORTED for a device index above 15).
 */
int mdls_init(void);
int mdls_finalize(void);

/*
 * Process-wide tuning, for benchmarks and tests; the defaults are built in and nothing is
 * read from the environment.  Only MDLS_TUNE_PANEL_VARIANT, MDLS_TUNE_SPLIT_UPDATE and
 * MDLS_TUNE_CPANEL change results (the panel's workgroup shape and so its reduction order; the
 * rounding of the update products; the complex reflector's formulas); the others change only
 * speed or, for the spin limit, how long a grid barrier (or the complex panel's wait for the
 * previous column) polls before it reports -1 through *d_info.
 *   MDLS_TUNE_LOOKAHEAD        1 (default): concurrent trailing update after mdls_init; 0: off
 *   MDLS_TUNE_PANEL_VARIANT    0 (default) or 1: the panel kernel's alternative shape (more rows
 *                              per thread: dd 512 x 8, qd 256 x 4, od 256 x 2 threads x rows);
 *                              octo-double factorisations of more than 1024 rows use the
 *                              alternative shape under either value
 *   MDLS_TUNE_APPLY_GRID_CAP   workgroups of the concurrent trailing update; 0 (default): 448
 *                              (two per CU on 224 CUs), for od 224 once fewer than
 *                              MDLS_TUNE_APPLY_WIDE_ROWS (default 768) rows remain
 *   MDLS_TUNE_SPIN_LIMIT       polls (each after a sleep of about 64 cycles) before a grid
 *                              barrier gives up; default 2^22
 *   MDLS_TUNE_SPLIT_UPDATE     0 (default) or 1: mdls_solve_refined's double-double factorisation
 *                              forms its trailing-update products Y^T C on the FP64 matrix cores
 *                              by exact slicing (the product of mdls_dd_gemm_tn method 1) instead
 *                              of on the vector units; the products are exactly rounded either
 *                              way up to the vector units' lazy accumulation, so results differ
 *                              only in the last bits of the factors
 *   MDLS_TUNE_CPANEL           the complex QR's tile panels: 0 one launch per panel column;
 *                              1 one persistent launch per panel (one workgroup per column, the
 *                              columns handed on through device memory); 2 (default) persistent
 *                              for qd and od, a launch per column for double and dd (the faster
 *                              form of each on MI355X).  The persistent form takes the reflector
 *                              scalars in another (equivalent) order, so results differ in the
 *                              last bits
 * mdls_set_tuning returns 0, -1 for an unknown option, -2 for a value out of range;
 * mdls_get_tuning returns the current value (-1 for an unknown option).
 */
enum {
    MDLS_TUNE_LOOKAHEAD = 1,
    MDLS_TUNE_PANEL_VARIANT = 2,
    MDLS_TUNE_APPLY_GRID_CAP = 3,
    MDLS_TUNE_APPLY_WIDE_ROWS = 4,
    MDLS_TUNE_SPIN_LIMIT = 5,
    MDLS_TUNE_SPLIT_UPDATE = 6,
    MDLS_TUNE_CPANEL = 7
};
int mdls_set_tuning(int option, long value);
long mdls_get_tuning(int option);

/* Largest number of rows the Householder panel kernel holds on chip, for precision p. */
int mdls_max_rows(int p);

/*
 * Bytes of device workspace that mdls_qr, mdls_apply_qt, mdls_backsub and mdls_solve need
 * for (p, m, n, tile).  The same workspace serves all four.  Returns 0 for invalid input.
 */
size_t mdls_workspace_bytes(int p, int m, int n, int tile);

/*
 * Householder QR (paper Section 3, Algorithm 2: inputs A, tile size and tile count; outputs R
 * and the blocked reflectors; the Householder vector and beta of each column as the paper
 * takes them from Golub and Van Loan, Algorithm 5.1.1).  A (m x n, lda >= m) is overwritten:
 * R in the upper triangle, the Householder vector v_j of column j below the diagonal (unit
 * first entry not stored), so R(j,j) >= 0 whenever the column below the diagonal is not
 * exactly zero, and beta_j = 0 with R(j,j) unchanged when it is.
 * beta (may be NULL): P planes of n, receives beta_0 .. beta_{n-1}.
 * T (may be NULL): P planes of ldt x n, ldt >= tile.  For each tile block k (columns
 * k*tile .. k*tile+tile-1) rows 0..tile-1 of those columns receive the upper-triangular
 * tile x tile factor T_k with H_{k*tile} ... H_{k*tile+tile-1} = I - Y_k T_k Y_k^T, Y_k the
 * unit lower trapezoidal block of Householder vectors; diag(T_k) holds the beta_j.
 * Deviation from the paper's output list: Algorithm 2 returns the W of P_WY = I + W Y^T
 * (Section 3, the recurrence for the columns of W) and the explicit Q; this call returns the
 * compact factor T instead, from which W_k = -Y_k T_k on request (mdls_form_w) and Q on
 * request (mdls_form_q), because Q^T b needs only Y and T (identical in exact arithmetic).
 * d_info (may be NULL): 0, or -1 if a grid barrier gave up (see the top of this file).
 * Requires n % tile == 0 when T != NULL, and m <= mdls_max_rows(p).  Status -1..-11 for
 * arguments 1..11.
 */
int mdls_qr(int p, int m, int n, int tile, double *A, int lda, double *beta, double *T, int ldt,
            void *ws, size_t ws_bytes, int *d_info, hipStream_t stream);

/*
 * B := Q^T B with Q = H_0 H_1 ... H_{n-1} from mdls_qr (paper Section 1: with A = QR the
 * system A x = b becomes R x = Q^T b; Section 3, the update with the blocked reflector).
 * A and T as returned by mdls_qr with the same tile.  B is m x nrhs (ldb >= m).  Applies the
 * tile blocks in order: B := (I - Y_k T_k^T Y_k^T) B, which is the paper's B + Y_k (W_k^T B)
 * with W_k = -Y_k T_k; it takes T where the paper's interface would take W (see mdls_qr).
 */
int mdls_apply_qt(int p, int m, int n, int tile, const double *A, int lda, const double *T,
                  int ldt, double *B, int ldb, int nrhs, void *ws, size_t ws_bytes,
                  hipStream_t stream);

/*
 * B := Q B (the tile blocks in reverse order: B := (I - Y_k T_k Y_k^T) B), and the explicit
 * orthogonal factor the paper's Algorithm 2 forms (Section 3): mdls_form_q writes the first
 * ncols (1 <= ncols <= m) columns of Q (m x m) into Q (P planes of ldq x ncols, ldq >= m).
 * A and T as returned by mdls_qr with the same tile; n % tile == 0.  Negative status as for
 * mdls_apply_qt (for mdls_form_q: -9 Q null, -10 ldq < m, -11 ncols, -12/-13 workspace).
 */
int mdls_apply_q(int p, int m, int n, int tile, const double *A, int lda, const double *T,
                 int ldt, double *B, int ldb, int nrhs, void *ws, size_t ws_bytes,
                 hipStream_t stream);
int mdls_form_q(int p, int m, int n, int tile, const double *A, int lda, const double *T,
                int ldt, double *Q, int ldq, int ncols, void *ws, size_t ws_bytes,
                hipStream_t stream);

/*
 * The paper's W factor (Section 3, eqs. for P_WY = I + W Y^T): W_k = -Y_k T_k for every
 * tile block, written to W (P planes of ldw x n, ldw >= m): block k occupies columns
 * k*tile.. and rows k*tile..m-1; rows above are set to zero.
 */
int mdls_form_w(int p, int m, int n, int tile, const double *A, int lda, const double *T,
                int ldt, double *W, int ldw, hipStream_t stream);

/*
 * Tiled back substitution (paper Section 2, Algorithm 1: input the N x N tiles of an upper
 * triangular U and b; output x with U x = b): solves R x = y with R the upper triangle of
 * the leading n x n block of R (ldr >= n, entries below the diagonal are not read), n a
 * multiple of tile.  x holds y on entry (P planes of n doubles) and the solution on exit.
 * Stage 1 inverts the n/tile diagonal tiles, stage 2 alternates x_i := U_i^{-1} b_i with
 * b_j -= A_{j,i} x_i for j < i.  *d_info: 0, or k > 0 for the first exactly zero R(k,k).
 */
int mdls_backsub(int p, int n, int tile, const double *R, int ldr, double *x, void *ws,
                 size_t ws_bytes, int *d_info, hipStream_t stream);

/*
 * Least squares (paper Section 1: the solution of A x = b in the least-squares sense via
 * A = QR and R x = Q^T b; Section 4, the least-squares runs time QR and back substitution
 * together): Algorithm 2 with Q^T b carried as an extra column of every trailing update, then
 * Algorithm 1 on R x = (Q^T b)(0:n).  A (m x n) and b (P planes of m) are overwritten by the
 * factors (as mdls_qr, without T) and by Q^T b, whose rows n..m-1 hold the residual's
 * coordinates; x (P planes of n) receives the solution.  tile is the back substitution tile
 * (n % tile == 0).  *d_info: 0; k > 0 for the first exactly zero R(k,k); -1 if a grid barrier
 * gave up.  Status -1..-11 for arguments 1..11.
 */
int mdls_solve(int p, int m, int n, int tile, double *A, int lda, double *b, double *x,
               void *ws, size_t ws_bytes, int *d_info, hipStream_t stream);

/*
 * mdls_solve without a workspace argument, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels, in the same order, with the same results bit for bit, but the workspace is a
 * static device array of MDLS_NOALLOC_SCRATCH_BYTES bytes inside the library, which each GPU
 * the library runs on holds until the process ends.  The call itself allocates nothing (no
 * hipMalloc, no stream, no event; launch timing is not recorded for it).  Its device address
 * is looked up once per device by mdls_init, or by the first call on a device if mdls_init was
 * not called there (make that first call outside graph capture).
 * Arguments as mdls_solve without ws and ws_bytes: -1..-9 for arguments 1..9 (d_info is
 * argument 9).  Returns MDLS_ESCRATCH when mdls_workspace_bytes(p, m, n, tile) exceeds
 * MDLS_NOALLOC_SCRATCH_BYTES (every square or tall n = 1024 solve fits, as does m = n = 2048
 * up to octo double).  Every call on one GPU shares that GPU's scratch and leaves its contents
 * behind (the solve clears what must start at zero itself): calls that overlap on one GPU, on
 * any streams or threads, race and give undefined results.
 */
#define MDLS_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int mdls_solve_noalloc(int p, int m, int n, int tile, double *A, int lda, double *b, double *x, int *d_info,
                       hipStream_t stream);

/* Static text for a status code. */
const char *mdls_status_string(int status);

/*
 * The double-double trailing-update product S = Y^T C (the GEMM-shaped update stage of
 * Algorithm 2, Section 3) on either execution unit, for the precision form's comparison:
 * method 0 runs it on the FP64 vector units in double-double arithmetic; method 1 on the FP64
 * matrix cores (MFMA) by exact slicing (Ozaki, Ogita, Oishi and Rump 2012): every column of Y
 * and C is scaled by a power of two, every entry cut into 7 slices of at most 19 bits, and
 * the slice products summed exactly in FP64 by level, then renormalised to double double
 * (normwise error below 2^-104 of max|Y| max|C| h).  Y is h x w (2 planes of ldy x w), C is
 * h x c (2 planes of ldc x c), S is w x c (2 planes of lds x c).  Method 1 needs h <= 2048
 * (the exactness bound), w <= 16, and a workspace of mdls_dd_gemm_tn_workspace_bytes(w, c)
 * bytes; method 0 needs none (ws may be NULL).  Status -1..-12 for arguments 1..12.
 */
size_t mdls_dd_gemm_tn_workspace_bytes(int w, int c);
int mdls_dd_gemm_tn(int method, int h, int w, int c, const double *Y, int ldy, const double *C,
                    int ldc, double *S, int lds, void *ws, size_t ws_bytes, hipStream_t stream);

/*
 * Complex least squares (the paper's complex workload: Section 3 replaces the transpose of
 * Algorithm 2 by the Hermitian transpose; Section 4, Table 5 times the complex double
 * double QR).  A complex matrix is 2P planes: the P limb planes of the real parts, then the
 * P limb planes of the imaginary parts (real and imaginary parts kept in separate arrays,
 * end of Section 2), each ld x cols column-major, plane stride ld * cols.  A complex vector
 * of length L is 2P planes of L doubles.  n must be a multiple of tile (1..256).  Ownership,
 * streams, errors and *d_info as for the real calls (d_info: R(k,k) with both parts exactly
 * zero); these calls use only the caller's stream.
 *
 * Householder vectors: for column x with x1 = |x1| e^{i theta} (theta = 0 when x1 = 0) and
 * sigma = sum_{i>1} |x_i|^2: sigma = 0 gives beta = 0 and R(j,j) = x1; otherwise mu =
 * sqrt(|x1|^2 + sigma), nu = -sigma/(|x1| + mu) (nu = -mu when x1 = 0), v1 = e^{i theta} nu,
 * beta = 2 nu^2/(sigma + nu^2) (real), v = x/v1 stored below the diagonal, and R(j,j) =
 * e^{i theta} mu -- Golub-Van Loan 5.1.1 on |x1|, rotated by the phase of x1, so that
 * H = I - beta v v^H is Hermitian and H x = R(j,j) e_1.
 */
size_t mdls_cworkspace_bytes(int p, int m, int n, int tile);

/*
 * Complex blocked Householder QR.  A (2P planes of lda x n) is overwritten with R (upper
 * triangle) and the v_j (below the diagonal, unit first entries not stored); beta stays in
 * the workspace.  T (may be NULL; 2P planes of ldt x n, ldt >= tile) receives for each tile
 * block k the upper-triangular T_k with H_{k*tile} ... H_{k*tile+tile-1} = I - Y_k T_k Y_k^H
 * (diag(T_k) = beta); the paper's W is W_k = -Y_k T_k.  Status -1..-10 for arguments 1..10.
 * A tile panel is one persistent launch (where MDLS_TUNE_CPANEL selects it) while its column
 * fits in 64 KiB of LDS (m - k*tile rows <= 4096/p) and its tile workgroups can all be
 * resident; a column waits for the one before it with a bounded poll: should a wait time out
 * (MDLS_TUNE_SPIN_LIMIT), R(0,0) is set to NaN here and mdls_csolve reports *d_info = -1.
 */
int mdls_cqr(int p, int m, int n, int tile, double *A, int lda, double *T, int ldt, void *ws,
             size_t ws_bytes, hipStream_t stream);

/*
 * B := Q^H B for the complex m x nrhs B (2P planes of ldb x nrhs), with A and T from mdls_cqr
 * (same tile): the tile blocks in order, B := (I - Y_k T_k^H Y_k^H) B.
 */
int mdls_capply_qh(int p, int m, int n, int tile, const double *A, int lda, const double *T,
                   int ldt, double *B, int ldb, int nrhs, void *ws, size_t ws_bytes,
                   hipStream_t stream);

/* B := Q B (the blocks in reverse, B := (I - Y_k T_k Y_k^H) B) and the first ncols columns of the
 * explicit unitary factor (2P planes of ldq x ncols), as mdls_apply_q and mdls_form_q for real data. */
int mdls_capply_q(int p, int m, int n, int tile, const double *A, int lda, const double *T,
                  int ldt, double *B, int ldb, int nrhs, void *ws, size_t ws_bytes,
                  hipStream_t stream);
int mdls_cform_q(int p, int m, int n, int tile, const double *A, int lda, const double *T,
                 int ldt, double *Q, int ldq, int ncols, void *ws, size_t ws_bytes,
                 hipStream_t stream);

/* Complex tiled back substitution (Algorithm 1): x (2P planes of n) holds y on entry and the
 * solution of R x = y on exit, R the upper triangle of the leading n x n block (ldr >= n). */
int mdls_cbacksub(int p, int n, int tile, const double *R, int ldr, double *x, void *ws,
                  size_t ws_bytes, int *d_info, hipStream_t stream);

/* Complex least squares: A and b (2P planes of m) are overwritten by the factors and Q^H b;
 * x (2P planes of n) receives the solution of R x = (Q^H b)(0:n). */
int mdls_csolve(int p, int m, int n, int tile, double *A, int lda, double *b, double *x,
                void *ws, size_t ws_bytes, int *d_info, hipStream_t stream);

/*
 * Batched least squares: many independent problems of uneven sizes solved in one
 * persistent launch (the paper's least-squares solve, Sections 2-3, per problem; its
 * uneven-size workloads, Section 4).  p is 2 (dd) or 4 (qd); every problem has
 * 1 <= n <= m <= 512.  Problem i's A is P planes of m x n (ld m, plane stride m n) at
 * A + a_off, its b P planes of m at b + b_off, its x P planes of n at x + x_off (offsets
 * in doubles).  A and b are overwritten (factors, Q^T b) as by mdls_solve.
 *
 *   mdls_batch_workspace_bytes(p, count)   workspace for a batch of count problems (0 if
 *                              p or count is invalid).
 *   mdls_batch_plan(p, count, h_desc, ws, ws_bytes, stream)
 *                              validates the HOST array h_desc and writes the processing
 *                              order (largest m n^2 first) into the workspace.  A set-up
 *                              call: it copies host to device and synchronises the stream,
 *                              so it must not be captured into a graph.  -3 if any
 *                              descriptor is invalid.
 *   mdls_solve_batched(p, count, A, b, x, variant, ws, ws_bytes, d_info, d_times, stream)
 *                              solves the planned batch: a counter reset and one persistent
 *                              kernel on `stream`, nothing else (graph-capturable; the
 *                              workspace keeps the plan).  variant selects the kernel shape
 *                              (0 <= variant < mdls_batch_variants(p)).  d_info (count device
 *                              ints) receives each problem's status as *d_info of
 *                              mdls_solve, or -1 if the workgroups sharing the problem timed
 *                              out at one of their barriers (x then unspecified; the largest
 *                              problems of a batch are shared by up to 16 workgroups, which
 *                              needs every workgroup of the launch resident at once, as it is
 *                              when nothing else occupies the GPU); d_times (2 count device
 *                              long longs, or null) the
 *                              start and end of each problem in wall-clock ticks
 *                              (mdls_wall_clock_khz).
 *   mdls_batch_variants(p)     number of kernel variants (0 if p is not supported).
 *   mdls_batch_autotune(p, count, A_src, b_src, a_len, b_len, A, b, x, ws, ws_bytes, d_info,
 *                       ms, stream)
 *                              the project's autotuner: for every variant, copies the pristine
 *                              A_src, b_src (a_len, b_len doubles) into A, b and times one
 *                              warm and one timed solve with events; ms (host, one float per
 *                              variant, or null) receives the times.  Synchronises the
 *                              stream.  Returns the fastest variant (>= 0) or a status < 0.
 *   mdls_wall_clock_khz(&khz)  tick rate of the d_times clock on the current device.
 */
typedef struct {
    int m, n;
    long long a_off, b_off, x_off;
} mdls_batch_desc;

/*
 * Refined least squares (the precision form): the accuracy of p_out = 4 (qd) or 8 (od) limbs
 * from a double-double factorisation.  A (m x n, double double, ld lda, read only) is copied
 * into F (same shape and ld, overwritten by its dd factors); Householder QR of F in dd with
 * the tile T factors (Section 3); then at most iters refinement steps with the residuals in
 * p_out limbs and the corrections in dd (Q^T and Q by the tile reflectors, R^-1 and R^-T by the
 * tiled back substitution of Section 2 and its transpose, with the tile inverses formed once):
 *   m == n: r := b - A x (x = 0 in the first step), d := R^-1 (Q^T r)(0:n), x += d;
 *   m > n: refinement of the augmented system [I A; A^T 0][r; x] = [b; 0] (Bjorck 1967), so
 *   that a nonzero residual does not limit the accuracy: r and x start at 0, and each step
 *   forms f := b - r - A x and g := -A^T r, then h := R^-T g, d := Q^T f,
 *   x += R^-1 (d(0:n) - h) and r += Q [h; d(n:m)].
 * b: P = p_out planes of m; x: p_out planes of n (output).  Each step gains about
 * -log10(kappa(A) 2^-105) digits while kappa(A) 2^-105 << 1.  iters is the most
 * steps taken: the call stops on the device once the correction norms show convergence, when
 * max|d| <= u max|x| or when the next correction estimated from the observed contraction,
 * d_k^2 / d_(k-1), is below u max|x| (u = 2^-(53 p_out - p_out + 1)); later steps' kernels then
 * return at once, so the call stays asynchronous and capturable.  d_norms (2 iters device
 * doubles) receives max |d| and max |x| (leading limbs) of each step taken and -1, -1 for
 * steps not taken.  *d_info as for mdls_solve.  n % tile == 0.
 *   mdls_refined_workspace_bytes(p_out, m, n, tile)   workspace (0 if arguments invalid).
 */
size_t mdls_refined_workspace_bytes(int p_out, int m, int n, int tile);
int mdls_solve_refined(int p_out, int m, int n, int tile, const double *A, int lda, const double *b,
                       double *x, int iters, double *F, void *ws, size_t ws_bytes, int *d_info,
                       double *d_norms, hipStream_t stream);

size_t mdls_batch_workspace_bytes(int p, int count);
int mdls_batch_plan(int p, int count, const mdls_batch_desc *h_desc, void *ws, size_t ws_bytes,
                    hipStream_t stream);
int mdls_solve_batched(int p, int count, double *A, double *b, double *x, int variant, void *ws,
                       size_t ws_bytes, int *d_info, long long *d_times, hipStream_t stream);
int mdls_batch_variants(int p);
int mdls_batch_autotune(int p, int count, const double *A_src, const double *b_src, size_t a_len,
                        size_t b_len, double *A, double *b, double *x, void *ws, size_t ws_bytes,
                        int *d_info, float *ms, hipStream_t stream);
int mdls_wall_clock_khz(int *khz);

/*
 * Per-kernel device timing, as the paper reports per-kernel times (Section 4, kernel time
 * versus wall time).  While enabled, every kernel the library launches is bracketed by two
 * HIP events recorded on the caller's stream, and recorded with its name, its precision P
 * and its algorithmic multiple-double multiply-add count.  Host-side state shared by all
 * threads of the process; meant for benchmarks, not for concurrent production calls.
 *   mdls_timing_enable(on)    start (on != 0) or stop recording; returns 0.
 *   mdls_timing_reset()       wait for and discard all records; returns 0, or MDLS_EHIP if a
 *                             recorded event could not be waited for.
 *   mdls_timing_query(name, p, &ms, &launches, &md_fmas)
 *                             waits for the recorded events and sums the launches of kernel
 *                             `name` ("" = all kernels) at precision p (0 = all); returns 0,
 *                             -i for a null argument i, MDLS_EHIP on an event error.
 *   mdls_timing_kernels(buf, len)
 *                             newline-separated names of the kernels recorded so far
 *                             (truncated to len - 1 bytes); returns the number of names.
 */
int mdls_timing_enable(int on);
int mdls_timing_reset(void);
int mdls_timing_query(const char *name, int p, double *total_ms, long *launches, double *md_fmas);
int mdls_timing_kernels(char *buf, int buflen);

#ifdef __cplusplus
}
#endif

#endif /* MDLS_H */
