/*
 * tdsolve -- series of symmetric tridiagonal systems on AMD Instinct MI355X
 * (gfx950), by the parallel sweep method of A.V. Terekhov, "Parallel
 * dichotomy algorithm for solving tridiagonal SLAEs" (arXiv:0901.2859).
 *
 * Problem (section 2, "Statement of the problem", eq. main_eq3):
 *     A X_n = F_n,  n = 1..N,
 * with one constant, symmetric, nondegenerate tridiagonal M x M matrix A:
 * diagonal b[0..M-1], off-diagonal a[0..M-2], A[i][i+1] = A[i+1][i] = a[i].
 * Non-symmetric tridiagonal matrices with A[i+1][i] A[i][i+1] > 0 are
 * reduced to this case by a diagonal similarity (section "Nonsymmetrical
 * matrices"; tdsolve_prepare_general).
 *
 * Method (section 3):
 *  - data decomposition (section 2): rows split into P contiguous blocks of
 *    at least 2 rows; the first M mod P blocks get one extra row;
 *  - preliminary step, once per matrix, in FP64 (Algorithm 3 step 1;
 *    Lemma 2, eq. green_v; eq. z_vector; Remark 1): the rows of A^{-1} at
 *    the P-1 interface rows (the first row of blocks 1..P-1) and the
 *    transfer factors of the vectors Z^R, Z^L between neighbouring
 *    interface rows;
 *  - per right-hand side (Algorithm 3 step 2): the weights beta^{R,L} of
 *    every block (eq. beta_symn), the interface components by the main
 *    parallel sweep theorem (Theorem 2, eq. theor_2, evaluated as two
 *    first-order recurrences over the blocks), then independent sweeps
 *    inside every block with its boundary values known (Lemma 1,
 *    Algorithm 1).
 *
 * Layout.  Every N-column array is RHS-interleaved, row-major [M][N]:
 * element (row i, right-hand side n) is at offset i*N + n.
 *
 * Precision modes (TDS_*):
 *   TDS_F64          F double, X double; FP64 sweeps.
 *   TDS_F32_REFINED  F float,  X double; FP32 sweeps inside each block with
 *                    FP64 interface values and FP64 residual-based
 *                    refinement passes, all in registers: `passes` passes
 *                    on the block's zero-boundary solution, then (passes >=
 *                    1) one more on the whole solution with its boundary
 *                    values (default 2 passes; blocks of more than 64 rows
 *                    are swept in FP64 arithmetic instead, as in
 *                    TDS_F32_WIDE).
 *   TDS_F32          F float,  X float;  FP32 sweeps, FP64 interface step.
 *   TDS_F32_WIDE     F float,  X double; FP64 sweeps of the widened input.
 *
 * Memory.  a, b are host arrays owned by the caller, copied by prepare.
 * F, X, gX, gF, ga, gb, and the output buffers of tdsolve_components and
 * tdsolve_residual are device pointers (the current HIP device) owned by
 * the caller.  X may equal F only when both have the same element type;
 * tdsolve_series and tdsolve_batch_series reject any other overlap of F and
 * X (TDS_EINVAL).  A handle owns its device tables and a
 * work buffer that grows with N; calls on one handle must be ordered on a
 * single stream (use one handle per concurrent stream).
 *
 * Errors.  Every entry point returns a tds_status code; no exception crosses
 * the ABI.  Launches are asynchronous on `stream` (a hipStream_t, NULL =
 * the default stream); a launch failure returns TDS_EHIP.
 */
#ifndef TDSOLVE_H
#define TDSOLVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tds_plan* tds_handle;

typedef enum {
    TDS_OK = 0,
    TDS_EINVAL = -1,        /* bad argument: sizes, null pointer, NaN/Inf in a or b */
    TDS_ESINGULAR = -2,     /* zero or non-finite pivot in the FP64 preliminary step */
    TDS_ENOMEM = -3,        /* host or device allocation failed */
    TDS_EHIP = -4,          /* a HIP runtime call or kernel launch failed */
    TDS_ENOCONV = -5,       /* reserved: refinement did not converge */
    TDS_EUNSUPPORTED = -6,  /* valid request outside what the library handles */
    TDS_ESCRATCH = -7       /* tdsolve_series_noalloc: the call's work area exceeds
                               the library's fixed 32 MiB scratch */
} tds_status;

typedef enum {
    TDS_F64 = 0,
    TDS_F32_REFINED = 1,
    TDS_F32 = 2,
    TDS_F32_WIDE = 3
} tds_mode;

/* Facts about a prepared matrix (host struct filled by tdsolve_info). */
typedef struct {
    int64_t M;            /* rows */
    int32_t P;            /* blocks */
    int32_t max_block;    /* largest block size t_j */
    int32_t dominant;     /* 1 if |b_i| >= |a_{i-1}| + |a_i| with one strict
                             inequality (Theorem 4's stability condition) */
    int32_t refine_passes;/* passes used by TDS_F32_REFINED */
    double max_ratio;     /* max |Z_{k+1}/Z_k| over both sweeps; <= 1 under
                             dominance (proof of Theorem 4) */
    int32_t general;      /* 1 for a plan of tdsolve_prepare_general */
    int32_t sweep_halves; /* 1 if the modes with FP64 results (TDS_F64,
                             TDS_F32_REFINED, TDS_F32_WIDE) sweep every block
                             in two halves (segments of 35..64 rows: a left
                             half of 32 interior rows, the middle row, the
                             rest) */
} tds_info;

/* Preliminary step (Algorithm 3 step 1).  a: M-1 host doubles (may be NULL
 * when M == 1), b: M host doubles.  P: number of blocks, 1 <= P <= M/2
 * (P == 1 allowed for any M >= 1); P == 0 picks a block count from the
 * library's size table.  On success *out receives a new handle.
 * Errors: TDS_EINVAL (sizes, NULL, non-finite a or b), TDS_ESINGULAR (an
 * elimination or ratio denominator is zero or non-finite in FP64),
 * TDS_ENOMEM, TDS_EHIP (device upload). */
int tdsolve_prepare(const double* a, const double* b, int64_t M, int32_t P,
                    tds_handle* out);

/* Preliminary step for a non-symmetric tridiagonal A (section
 * "Nonsymmetrical matrices"): row i reads lower[i-1] x_{i-1} + diag[i] x_i +
 * upper[i] x_{i+1} (lower, upper: M-1 host doubles, A[i+1][i] = lower[i],
 * A[i][i+1] = upper[i]; NULL allowed when M == 1).  Requires
 * lower[i] * upper[i] > 0 for every i: then the diagonal similarity
 * D^{-1} A D with d_{i+1} / d_i = sqrt(lower[i] / upper[i]) is symmetric and
 * the symmetric preliminary step applies to it; the weights and transfer
 * factors are mapped back to A, and the block sweeps run on A itself, so
 * tdsolve_series, tdsolve_components and tdsolve_residual work unchanged.
 * tdsolve_backward returns TDS_EUNSUPPORTED for such a plan (its adjoint
 * solves with A^T).  Errors: as tdsolve_prepare, and TDS_EUNSUPPORTED when
 * some lower[i] * upper[i] <= 0. */
int tdsolve_prepare_general(const double* lower, const double* diag,
                            const double* upper, int64_t M, int32_t P,
                            tds_handle* out);

/* Solve the series (Algorithm 1 with Algorithm 3 step 2 for the interface
 * rows).  F: device [M][N] (double for TDS_F64, float otherwise).
 * X: device [M][N] (float for TDS_F32, double otherwise).  X may be F
 * itself when both have the same element type; any other overlap of the
 * two arrays is TDS_EINVAL.  N >= 0 (N == 0 is a no-op; TDS_EUNSUPPORTED
 * when N / 16 exceeds the launch grid, 2^31 - 1).  Asynchronous on
 * `stream`. */
int tdsolve_series(tds_handle h, const void* F, void* X, int64_t N,
                   int32_t mode, void* stream);

/* tdsolve_series without any device allocation, for callers that cannot
 * allocate: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, checks, kernels and results
 * (bitwise) as tdsolve_series on the same plan, but the per-right-hand-side
 * work area (beta^R, beta^L: P x N doubles each; the interface values:
 * (P-1) x N doubles; with TDS_IFACE_DICHOTOMY two more (P+1) x N; the
 * counters of the fused order, 2 + 2 ceil(N / 256) lines of 256 bytes;
 * every slice rounded up to 256 bytes) comes from a fixed 32 MiB device
 * array of the library instead of the plan's work buffer: N <= 10943 at
 * P = 128, N <= 21930 at P = 64 (the recurrence and dense orders).  A larger request returns TDS_ESCRATCH
 * before anything is launched.  The call allocates nothing (no hipMalloc,
 * no hipFree, no host allocation); the array's address on the current
 * device is looked up once, on the first call on that device.  The plan
 * must have been prepared on the current device (else TDS_EINVAL).  Every
 * call on one GPU shares that GPU's array: calls that overlap in time on
 * one GPU (concurrent streams, threads) race and must not be issued.  The
 * call is not recorded for tdsolve_status and takes no phase timing. */
int tdsolve_series_noalloc(tds_handle h, const void* F, void* X, int64_t N,
                           int32_t mode, void* stream);

/* Algorithm 3 alone: the solution components at the P-1 interface rows for
 * every right-hand side, without the block sweeps.  Xsep: device double
 * [P-1][N]; row k-1 holds x at the first row of block k.  F as for
 * tdsolve_series (mode selects the element type of F only). */
int tdsolve_components(tds_handle h, const void* F, double* Xsep, int64_t N,
                       int32_t mode, void* stream);

/* Adjoint of X = A^{-1} F for a loss L with dL/dX = gX (device [M][N],
 * same element type as X of `mode`).  Since A is symmetric (Lemma 2), the
 * same prepared plan gives gF = A^{-1} gX (written to gF, same element type
 * as F of `mode`).  ga (M-1 doubles) and gb (M doubles), device pointers,
 * are overwritten with dL/da and dL/db:
 *   gb_i = -sum_n gF[i][n] X[i][n],
 *   ga_i = -sum_n (gF[i][n] X[i+1][n] + gF[i+1][n] X[i][n]).
 * Either may be NULL to skip it.  X: device [M][N] forward solution (same
 * element type as gX).  Reductions are in a fixed order (bitwise
 * reproducible). */
int tdsolve_backward(tds_handle h, const void* X, const void* gX, void* gF,
                     double* ga, double* gb, int64_t N, int32_t mode,
                     void* stream);

/* Residual check of a computed solution: for every right-hand side n,
 * out[n] = ||F_n - A X_n||_inf / (||A||_inf ||X_n||_inf + ||F_n||_inf)
 * (normwise backward error) and out[N + n] = ||F_n - A X_n||_2 / ||F_n||_2.
 * F, X as for tdsolve_series with `mode`; out: device double [2N]. */
int tdsolve_residual(tds_handle h, const void* F, const void* X, int64_t N,
                     int32_t mode, double* out, void* stream);

/* Per-phase timing for measurement.  While enabled, every tdsolve_series
 * and tdsolve_batch_series call on the handle launches its three kernels
 * with start and stop events (hipExtLaunchKernelGGL), which take each
 * kernel's own start and end timestamps: the phases exclude the dispatch
 * gaps between kernels.  tdsolve_timing_read waits for the last recorded
 * event, writes the accumulated milliseconds of [0] the beta weights,
 * [1] the interface step and [2] the block sweeps into ms (3 host doubles)
 * and the number of timed calls into *calls, then clears the record.  Keep
 * timing off while a stream is being captured into a graph. */
/* Status of the handle's last series solve: an a-posteriori check of the
 * accuracy the method guarantees for diagonally dominant A (Theorem 4).
 * Synchronises `stream`, recomputes the residuals of the last
 * tdsolve_series call (of every matrix of the last tdsolve_batch_series
 * call, for a batch handle) from that call's F and X, which must still hold
 * its input and result, and writes to *backward_err the largest normwise
 * backward error max_n ||F_n - A X_n||_inf / (||A||_inf ||X_n||_inf +
 * ||F_n||_inf) (NaN if any right-hand side gave a non-finite value; 0 for
 * an empty call), and to *passes the refinement passes that call used (0
 * unless TDS_F32_REFINED).  Either output may be NULL.  Allocates and frees
 * a scratch buffer of about 5 M N / 64 doubles.  Errors: TDS_EINVAL (NULL
 * handle, or no series call on it yet), TDS_ENOMEM, TDS_EHIP. */
int tdsolve_status(tds_handle h, void* stream, double* backward_err,
                   int32_t* passes);

int tdsolve_timing_enable(tds_handle h, int32_t on);
int tdsolve_timing_read(tds_handle h, double* ms, int64_t* calls);

/* Evaluation order of the interface values (Algorithm 3 step 2.2) for
 * tdsolve_series and tdsolve_components of a single-matrix plan:
 *   TDS_IFACE_RECURRENCE (default): Theorem 2's sums as two first-order
 *     recurrences over the interface rows, O(P) per right-hand side;
 *   TDS_IFACE_DICHOTOMY: Algorithm 4 (Theorem 3, eq. omega_i): the
 *     interface rows level by level, each from its nearest known
 *     neighbours, rows of one level in parallel; O(P log P) per
 *     right-hand side and a work area of 2 (P + 1) N doubles more;
 *   TDS_IFACE_DENSE: Theorem 2's double sum (eq. theor_2) as one dense
 *     product, Xsep = K [beta^R; beta^L], on the FP64 matrix cores, with
 *     K ((P-1) x 2P: the ratio products between interface rows) built by
 *     the call in FP64 and uploaded (about 16 P^2 bytes of device memory,
 *     held until tdsolve_destroy); O(P^2) per right-hand side.  P <= 1024,
 *     else TDS_EUNSUPPORTED; the call allocates and copies synchronously.
 * All give the same values up to rounding.  TDS_EINVAL for other values or
 * a batch handle; TDS_ENOMEM / TDS_EHIP if the dense table cannot be
 * allocated or uploaded (the order is then unchanged). */
enum { TDS_IFACE_RECURRENCE = 0, TDS_IFACE_DICHOTOMY = 1, TDS_IFACE_DENSE = 2 };
int tdsolve_set_interface(tds_handle h, int32_t order);

/* Fused order of the per-right-hand-side step for tdsolve_series and
 * tdsolve_series_noalloc of a single-matrix plan.  lag == 0 (default): three
 * launches over the whole series (beta weights, interface values, block
 * sweeps).  lag >= 1: one launch (after a small one that clears its
 * counters) whose workgroups take the work items in ticket order, tile by
 * tile of `tile` right-hand sides (a multiple of 256, at most 2^20): the
 * beta weights of a tile, `lag` tiles later its interface values (each
 * waits until the tile's weights are published), `lag` tiles later still
 * its block sweeps (each waits for its tile's interface values only after
 * its zero-boundary solves).  Reads of F
 * for the weights overlap the writes of X, and the sweeps reread their F
 * soon after the weights did.  Same work items and arithmetic as the three
 * launches: bitwise the same X.  Taken when the plan sweeps its blocks in
 * halves (tdsolve_info.sweep_halves), the mode has FP64 results, the order
 * is the recurrence or the dense one, N is even and F is 8-byte (FP32
 * input) or 16-byte (FP64 input) aligned; otherwise the three launches
 * run.  Phase timing then reports the fused kernel as the sweep phase.
 * Errors: TDS_EINVAL (batch handle, lag outside 0..64, a bad tile). */
int tdsolve_set_fused(tds_handle h, int32_t lag, int32_t tile);

/* Number of refinement passes for TDS_F32_REFINED (0..8; default 2): FP64
 * residual passes on each block's zero-boundary solution; with 1 or more, a
 * last pass follows on the solution with its boundary values. */
int tdsolve_set_refinement(tds_handle h, int32_t passes);

int tdsolve_info(tds_handle h, tds_info* info);

/* Host-only copy of the preliminary step's FP64 tables, for checks without
 * a GPU.  Any output pointer may be NULL.  Sizes: starts P+1 (int64),
 * wR, wL: M (row i of segment j holds (A^{-1})[s_{j+1}][i] in wR and
 * (A^{-1})[s_j][i] in wL, 0 where undefined), rho, lam: P (rho[k], lam[k]
 * for k = 1..P-2 link interface rows k and k+1; other entries 0),
 * diag_inv: M (the diagonal of A^{-1}).  Same errors as prepare except
 * TDS_EHIP / device errors, which cannot occur. */
int tdsolve_prepare_host(const double* a, const double* b, int64_t M,
                         int32_t P, int64_t* starts, double* wR, double* wL,
                         double* rho, double* lam, double* diag_inv);

/* The same tables for a non-symmetric A (as tdsolve_prepare_general):
 * wR, wL are rows of A^{-1} at the interface rows, rho, lam the transfer
 * factors of the solution between neighbouring interface rows. */
int tdsolve_prepare_host_general(const double* lower, const double* diag,
                                 const double* upper, int64_t M, int32_t P,
                                 int64_t* starts, double* wR, double* wL,
                                 double* rho, double* lam, double* diag_inv);

/* Host-only copy of the coefficients of TDS_IFACE_DENSE (Theorem 2,
 * eq. theor_2, as one matrix), for checks without a GPU.  K receives
 * (P-1) x 2P doubles, row-major: for the interface row k = 1..P-1, row k-1
 * holds at column j < k the ratio product Z^R(s_{j+1}, s_k) =
 * rho_{j+1} ... rho_{k-1} (the weight of beta^R_j) and at column P + j,
 * j >= k, Z^L(s_j, s_k) = lam_k ... lam_{j-1} (the weight of beta^L_j);
 * every other entry is 0.  2 <= P <= 1024 (else TDS_EINVAL /
 * TDS_EUNSUPPORTED); other errors as tdsolve_prepare_host. */
int tdsolve_dense_table_host(const double* a, const double* b, int64_t M,
                             int32_t P, double* K);

/* Block count the library would choose for P == 0. */
int32_t tdsolve_default_blocks(int64_t M);

/* Measured block count.  The split into P blocks is free in the method
 * (Algorithm 3 holds for any P with blocks of >= 2 rows); it trades the
 * interface work per right-hand side, which grows with P, against the
 * block sweeps, whose register footprint grows with the rows per block.
 * Times tdsolve_series for blocks of at most 16, 32, 64 and 128 rows (and
 * P = 1 when M <= 128) on N device-generated uniform[-1, 1) right-hand
 * sides in `mode`, `reps` timed calls each (<= 0: 5), and writes the
 * fastest P to *P_out and its milliseconds per call to *ms_out (may be
 * NULL).  a, b as for tdsolve_prepare.  Allocates and frees device memory
 * and synchronises `stream`.  Errors: as tdsolve_prepare, TDS_EINVAL for
 * N < 1 or a bad mode, TDS_ENOMEM, TDS_EHIP. */
int tdsolve_autotune(const double* a, const double* b, int64_t M, int64_t N,
                     int32_t mode, int32_t reps, int32_t* P_out, double* ms_out,
                     void* stream);

/* A measured configuration of a single-matrix plan (tdsolve_autotune_plan). */
typedef struct {
    int32_t P;          /* block count */
    int32_t order;      /* TDS_IFACE_RECURRENCE or TDS_IFACE_DENSE */
    int32_t passes;     /* refinement passes for TDS_F32_REFINED (else 0) */
    int32_t fuse_lag;   /* tdsolve_set_fused lag (0: three launches) */
    int32_t fuse_tile;  /* tdsolve_set_fused tile */
    int32_t pad_;
    double ms;          /* milliseconds per solve of the choice */
    double r2;          /* largest relative residual ||F - A X||_2 / ||F||_2 of
                           the choice on the timing right-hand sides */
} tds_tuning;

/* Measured plan configuration for series of N right-hand sides in `mode`:
 * the block count (P == 0: blocks of at most 16, 32, 64 or 128 rows, and
 * P = 1 for M <= 128; P > 0: that count), the interface order (recurrence,
 * or the dense product for P <= 1024) and the fused order (three launches,
 * or one launch with lag 8 over tiles of 512 right-hand sides, for plans
 * that sweep in halves) are timed on F (device [M][N] of the mode's input
 * type; NULL: device-generated uniform[-1, 1) values), each candidate in
 * three interleaved rounds of `reps` calls (<= 0: 5), keeping its fastest
 * round.  For TDS_F32_REFINED the refinement passes of each block count are
 * fixed first, by accuracy: the fewest (1..3) whose largest relative
 * residual on F is within 1.25 times that of the same plan's TDS_F32_WIDE
 * solve (FP64 arithmetic).  Allocates and frees device memory and synchronises
 * `stream`.  Errors: as tdsolve_prepare, TDS_EINVAL (N < 1, P < 0, bad mode,
 * NULL out), TDS_ENOMEM, TDS_EHIP. */
int tdsolve_autotune_plan(const double* a, const double* b, int64_t M, int64_t N,
                          int32_t mode, int32_t P, const void* F, int32_t reps,
                          tds_tuning* out, void* stream);

int tdsolve_destroy(tds_handle h);

const char* tdsolve_strerror(int code);

/* ---- uneven batches: K independent matrices in one launch sequence ----
 * Each matrix k has its own a[k] (M[k]-1 doubles), b[k] (M[k] doubles),
 * block count P[k] (0 = library choice) and series of N[k] right-hand
 * sides.  The batch handle owns the concatenated tables of all K plans. */
int tdsolve_batch_prepare(int32_t K, const double* const* a,
                          const double* const* b, const int64_t* M,
                          const int32_t* P, tds_handle* out);

/* F[k], X[k]: device pointers of matrix k's [M[k]][N[k]] arrays (element
 * types by `mode` as for tdsolve_series); the pointer arrays themselves are
 * host arrays of K entries.  N: host array of K counts (0 allowed).  All K
 * series are solved by one launch of each kernel.  The per-matrix work
 * descriptors are uploaded only when pointers or counts differ from the
 * previous call or the one-launch lag (tdsolve_batch_set_fused) changed,
 * which synchronises `stream` (a host-to-device copy);
 * repeating a call with the same arguments issues kernel launches only, so
 * it can be captured in a HIP graph after one uncaptured call.
 * Errors: TDS_EINVAL (null arrays or pointers, N[k] < 0, F[k] == X[k] with
 * different element types), TDS_EUNSUPPORTED (more work items than one
 * launch holds), TDS_ENOMEM, TDS_EHIP. */
int tdsolve_batch_series(tds_handle hb, const void* const* F, void* const* X,
                         const int64_t* N, int32_t mode, void* stream);

/* One-launch order of tdsolve_batch_series (the steps of Algorithm 3 for
 * every matrix of the batch in one grid).  lag == 0 (default): the launches
 * of tdsolve_batch_series.  lag >= 1: one launch (after a small one that
 * clears its counters) whose workgroups take the work items of all
 * matrices in ticket order, two per ticket, tile by tile of 256 right-hand
 * sides of each matrix in turn: the beta weights of tile s, the interface
 * values of tile s - lag (each waiting until the weights of its tile are
 * published) and the block sweeps of tile s - 2 lag (each waiting until
 * its tile's interface values are published).  Waits are only on earlier
 * items and bounded.  Same work items and arithmetic as the separate launches:
 * bitwise the same X.  Taken when every matrix with right-hand sides has
 * blocks of at most 32 rows; otherwise the separate launches run.  Its
 * ticket table (8 bytes per work item) is uploaded with the descriptors,
 * and its counters (2 + 2 T lines of 256 bytes for T tiles) sit in the
 * handle's work buffer.  Phase timing reports the launch as the sweep
 * phase.  Errors: TDS_EINVAL (not a batch handle, lag outside 0..64). */
int tdsolve_batch_set_fused(tds_handle hb, int32_t lag);

/* Measured block counts for a batch.  Each matrix gets 32 or 64 rows per
 * block (P[k] = ceil(M[k] / rows) within the method's limits; the batch
 * runs one launch of each kernel per register row bucket, and with 64 rows
 * the sweeps take the blocks in halves).  First the same rows for every
 * matrix, both choices timed on tdsolve_batch_series with N[k]
 * device-generated right-hand sides in three interleaved rounds; then the
 * matrices in four classes of equal count by M[k] N[k], largest first: each
 * class's rows are flipped and kept when the batch is faster (the current
 * and the flipped batch timed in alternation).  The chosen P[k] go to P_out
 * (K entries), the milliseconds per call to *ms_out (may be NULL).  For
 * TDS_F32_REFINED, *passes_out (may be NULL; 0 in other modes) receives the
 * fewest refinement passes (1..3) whose largest normwise backward error
 * (tdsolve_status) stays within 1.25 times that of the same batch solved in
 * FP64 arithmetic (TDS_F32_WIDE).  Last, the launch order: the one-launch
 * order (tdsolve_batch_set_fused) at lags 8, 16 and 32 with 32 rows per
 * block for every matrix, against the chosen blocks in separate launches,
 * timed in interleaved rounds (for TDS_F32_REFINED only when the chosen
 * blocks are all 32-row ones, with the chosen passes).  When the one launch
 * is faster, P_out holds the 32-row blocks and *lag_out (may be NULL) its
 * lag; otherwise *lag_out is 0.  *ms_out: milliseconds per call of the
 * chosen configuration.  Allocation, synchronisation and errors as
 * tdsolve_autotune. */
int tdsolve_batch_autotune(int32_t K, const double* const* a,
                           const double* const* b, const int64_t* M,
                           const int64_t* N, int32_t mode, int32_t reps,
                           int32_t* P_out, int32_t* passes_out, int32_t* lag_out,
                           double* ms_out, void* stream);

/* Scaled strided copy dst = alpha * src of an S x M x L array of doubles
 * (f64 != 0) or floats, for the drivers that move the series between a
 * mesh layout and the RHS-interleaved layout (section "Variable separation
 * method": the harmonics of S problems become one series per harmonic).
 * Element (s, i, l) lives at src[s*ss[0] + i*ss[1] + l*ss[2]] and
 * dst[s*ds[0] + i*ds[1] + l*ds[2]] (device pointers; strides in elements,
 * host arrays of 3, non-negative).  Tiled through LDS per i, so a copy that
 * is contiguous along l on one side and along s on the other (a transpose)
 * reads and writes whole rows.  src and dst must not overlap.
 * Errors: TDS_EINVAL (null pointers with a non-empty array, negative sizes
 * or strides), TDS_EUNSUPPORTED (M > 65535), TDS_EHIP. */
int tdsolve_strided_copy(const void* src, void* dst, int32_t f64, int64_t S, int64_t M,
                         int64_t L, const int64_t* ss, const int64_t* ds, double alpha,
                         void* stream);

#ifdef __cplusplus
}
#endif

#endif /* TDSOLVE_H */
