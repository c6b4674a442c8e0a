/*
 * tileqr: tile Householder QR for MI355X (gfx950), FP64, with an empirical
 * (NB, IB) autotuner and a learned cost model.
 *
 * The method is the tile QR factorization of Section 2.1 of Agullo, Dongarra,
 * Nath and Tomov, "A Fully Empirical Autotuned Dense QR Factorization for
 * Multicore Architectures": the matrix is cut into tiles of order NB and
 * factorized by a DAG of four kernels (DGEQRT, DTSQRT, DLARFB, DSSRFB); the
 * inner blocking IB trades memory traffic for extra flops (Section 2.2). The
 * pair (NB, IB) is the tunable of Problem 2.1, chosen at run time from a
 * decision table built at install time by the two-step empirical search of
 * Sections 4-6 (qr_tune).
 *
 * Conventions for every entry point:
 *  - Matrices are FP64, column-major, with an explicit leading dimension.
 *    Pointers named A, T, B, X, y, params, grad are DEVICE pointers unless
 *    the comment says host. The caller allocates and owns every buffer; the
 *    library never frees caller memory. The library keeps only internal
 *    state (cached task lists, dependency counters, captured graphs, the
 *    decision table, the cost model, the compute-unit setting), process-wide
 *    and released at process exit.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Device work is enqueued asynchronously on it; the return code covers
 *    argument checking and launch errors. qr_sync() reports errors found by
 *    the device (a dependency wait that exceeded the watchdog).
 *  - Return codes follow LAPACK's info: 0 success; -i: argument i (1-based)
 *    is invalid; positive: TILEQR_ERR_* below.
 *  - QR has no numerical failure: rank deficiency gives zero diagonal
 *    entries in R; NaN/Inf propagate unchecked.
 *  - Range: a reflector's norm is formed from the unscaled sum of squares of
 *    its column (no LAPACK-style rescaling), so entries must stay within
 *    about 1e-150 .. 1e150 in magnitude: above it the sum overflows, below it
 *    a nonzero tail can round to a zero norm and be left in place. Scale the
 *    matrix first when its entries may leave that range.
 */
#ifndef TILEQR_H
#define TILEQR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TILEQR_OK 0
#define TILEQR_ERR_HIP 1         /* a HIP runtime call failed                  */
#define TILEQR_ERR_WATCHDOG 2    /* device scheduler wait timed out (qr_sync)   */
#define TILEQR_ERR_NOMEM 3       /* internal device allocation failed          */
#define TILEQR_ERR_NODEVICE 4    /* no usable gfx950 device                    */
#define TILEQR_ERR_TOO_LARGE 5   /* tile DAG too large (more than 2^31 tasks)  */
#define TILEQR_ERR_INTERNAL 6    /* plan construction failed (a library bug)   */
#define TILEQR_ERR_NOTABLE 7     /* decision table file missing or malformed   */
#define TILEQR_ERR_DISABLED 8    /* NB above the largest enabled tile class    */

/* Library version string (host, static storage). */
const char *qr_version(void);

/* ---------------------------------------------------------------------- */
/* Factorization (Section 2.1: tile QR as a DAG of GEQRT/TSQRT/LARFB/SSRFB) */
/* ---------------------------------------------------------------------- */

/* Number of doubles the T buffer of qr_factor needs:
 *   KT * MT * IB * NB,  MT = ceil(M/NB), NT = ceil(N/NB), KT = min(MT, NT).
 * T of tile (i, k) (i >= k, k < KT) is the IB x nb_k array at offset
 * (k*MT + i) * IB * NB with leading dimension IB; its column block
 * [s, s+IB) holds the upper-triangular compact-WY factor T_s of reflectors
 * s..s+IB-1 of that tile (Schreiber-Van Loan form: H_s ... H_{s+IB-1} =
 * I - V_s T_s V_s^T). Host only. Returns the size, or -1..-4 for an invalid
 * argument (same numbering as below: M, N, NB, IB). NB or IB of 0 is invalid
 * here (resolve them with qr_tune first). */
int64_t qr_T_size(int64_t M, int64_t N, int NB, int IB);

/* A = Q R for an M x N matrix (any M, N >= 0; ragged edge tiles allowed).
 *  A   (in/out, device, lda >= max(1, M)): on exit R is in the upper
 *      triangle/trapezoid; below it, tile by tile, the Householder vectors:
 *      in diagonal tiles unit-lower (unit implicit) as in DGEQRT, in tiles
 *      (i, k), i > k, the full vectors of DTSQRT.
 *  NB  tile order, 16 <= NB <= 512; IB inner block, 1 <= IB <= NB (IB need
 *      not divide NB: the last block of a tile is narrower). NB = 0 or IB = 0:
 *      taken from qr_tune(M, N, 1). The
 *      persistent grid is sized for qr_tune_units(M, N, 1) compute units.
 *  T   (out, device, qr_T_size(M, N, NB, IB) doubles): the T factors.
 * One persistent kernel runs the whole DAG; the dependency counters and the
 * task order are library state, so calls on the same device must not
 * overlap in time (enqueue them on one stream). Errors: -1 A null (with
 * M*N > 0), -2 M < 0, -3 N < 0, -4 lda < max(1, M), -5 NB, -6 IB, -7 T null. */
int qr_factor(double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, double *T,
              void *stream);

/* qr_factor for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same arguments, errors and results (A and T bit-identical to qr_factor's),
 * but no hipMalloc, hipFree or other allocating call. Its dependency counters,
 * ticket and error word live in a static device array of 16 MiB per device
 * (4 Mi ints), looked up on the first call on a device; the DAG runs in the
 * sequential program order of the tile algorithm, decoded on the device from
 * each ticket, so no task list is stored (and no list schedule is used: it
 * is slower than qr_factor). TILEQR_ERR_TOO_LARGE when the counters
 * (min(MT,NT)*MT + MT*NT*ceil(NB/strip) ints, strip = 64/32/16 columns for
 * NB <= 128/256/512) exceed the array. Every call on a device shares that
 * device's array, which keeps the last call's contents: calls that overlap
 * on one device (on different streams) race. The array is cleared by a
 * kernel at each call (no memset node). Watchdog errors are reported by
 * qr_sync. */
int qr_factor_noalloc(double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, double *T,
                      void *stream);

/* B <- Q^T B with Q from qr_factor(A, M, N, lda, NB, IB, T). NB and IB must
 * be the ones the factorization used (V and T depend on them); 0 resolves
 * through qr_tune(M, N, 1) as in qr_factor, which reproduces its choice as
 * long as the decision table and model are unchanged in between. B is
 * M x nrhs with ldb >= max(1, M); A and T are read only.
 * Errors: -1 A, -2 M, -3 N, -4 lda, -5 NB, -6 IB, -7 T, -8 B null,
 * -9 nrhs < 0, -10 ldb. */
int qr_apply_Qt(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB,
                const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream);

/* Communication-avoiding variant (Section 7: the tile rows split into p
 * domains, each reduced by its own GEQRT + TSQRT chain, the domains' R
 * factors merged pairwise over a binary tree), so the panel of a tall matrix
 * is reduced in parallel instead of by one chain of MT tasks. p = 1 is the
 * flat tree of qr_factor (same results bit for bit); p = 0 takes the decision
 * table's domain count; p > MT is taken as MT (one tile row per domain). The
 * domains hold h = ceil(MT / p) consecutive tile rows.
 *  A   (in/out): R in the upper triangle/trapezoid as in qr_factor; below
 *      it the reflectors of the domains' GEQRT (unit-lower part of each
 *      domain's first tile) and TSQRT (full tiles); the upper parts of the
 *      domains' first tiles below the diagonal hold their R before merging.
 *  T   (out, device, qr_T_size_ca(M, N, NB, IB, p) doubles): the per-tile T
 *      factors as in qr_factor, then the merges' reflector blocks
 *      (min(MT,NT) x domains blocks of NB x NB) and their T factors.
 * Errors as qr_factor with p in position 7: -7 p < 0, -8 T null. */
int64_t qr_T_size_ca(int64_t M, int64_t N, int NB, int IB, int p);
int qr_factor_ca(double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p, double *T,
                 void *stream);

/* B <- Q^T B with Q from qr_factor_ca(A, M, N, lda, NB, IB, p, T) (the same
 * NB, IB and p). Errors as qr_apply_Qt with p in position 7: -7 p < 0,
 * -8 T, -9 B, -10 nrhs, -11 ldb. */
int qr_apply_Qt_ca(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p,
                   const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream);

/* ---------------------------------------------------------------------- */
/* On top of (V, T): Q itself, B <- Q B, least squares (Section 2.1: Q is */
/* the product of the block reflectors the factorization stored)          */
/* ---------------------------------------------------------------------- */

/* B <- Q B with Q from qr_factor_ca(A, M, N, lda, NB, IB, p, T) (p = 1:
 * qr_factor): the reflectors of the Q^T application in the opposite order,
 * each block reflector I - V T V^T instead of its transpose. Arguments and
 * errors as qr_apply_Qt_ca (qr_apply_Q: as qr_apply_Qt, flat tree). */
int qr_apply_Q_ca(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p,
                  const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream);
int qr_apply_Q(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB,
               const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream);

/* The first k columns of Q (0 <= k <= M) explicitly: Q (out, device, M x k,
 * ldq >= max(1, M)) <- Q [I_k; 0]. A and T as in qr_apply_Q_ca. Errors as
 * qr_apply_Q_ca for A .. T, then -9 Q null (with M*k > 0), -10 k, -11 ldq. */
int qr_form_Q_ca(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p,
                 const double *T, double *Q, int64_t k, int64_t ldq, void *stream);

/* Least squares min ||A X - B|| for M >= N from the factorization: B (in/out,
 * device, M x nrhs, ldb >= max(1, M)) <- Q^T B, then its first N rows <-
 * R^-1 (Q^T B)[0:N] (back substitution with the upper triangle of A, one
 * workgroup per right-hand side). On exit rows 0..N-1 of B hold X and rows
 * N..M-1 the residual's coordinates Q^T (B - A X) (their norm is the
 * residual norm). A rank-deficient R (a zero diagonal entry) gives Inf/NaN.
 * Errors as qr_apply_Qt_ca; -3 also for N > M. */
int qr_solve_ls_ca(const double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, int p,
                   const double *T, double *B, int64_t nrhs, int64_t ldb, void *stream);

/* Many independent factorizations of uneven sizes in ONE persistent launch
 * over the union of their DAGs, each matrix with its own (NB, IB); the
 * launch is captured in a hipGraph the first time a given batch (pointers,
 * sizes, tile shapes) is seen and replayed afterwards.
 *  A, M, N, lda, NB, IB, T: HOST arrays of length count (A[b], T[b] device
 *  pointers; T[b] sized by qr_T_size). NB[b] = 0 or IB[b] = 0: from
 *  qr_tune(M[b], N[b], count). All NB[b] in one call share the register
 *  class of the largest (<= 64, <= 128, <= 256, <= 512).
 * Errors: -1 A, -2 M, -3 N, -4 lda, -5 count < 0, -6 NB, -7 IB, -8 T
 * (first offending entry). */
int qr_factor_batched(double *const *A, const int64_t *M, const int64_t *N, const int64_t *lda,
                      int64_t count, const int *NB, const int *IB, double *const *T, void *stream);

/* Same arguments and results as qr_factor_batched, but as a loop of one
 * qr_factor launch per matrix on the stream (the baseline the batched
 * launch is compared with). */
int qr_factor_loop(double *const *A, const int64_t *M, const int64_t *N, const int64_t *lda,
                   int64_t count, const int *NB, const int *IB, double *const *T, void *stream);

/* Sizes the persistent grid, and the schedule the host builds for it, for
 * `cus` compute units in the launches that follow (the device's count: all
 * of them; 0: no setting, the decision table's units decide, see
 * qr_tune_units): the setting for a stream created with a compute-unit mask
 * (hipExtStreamCreateWithCUMask) of that many units, or a smaller grid on
 * the whole device; the analog of the core count of Sections 4-6. Errors:
 * -1 cus < 0 or above the device's count; positive: no device. */
int qr_set_compute_units(int cus);

/* Waits for the stream, then returns (and clears) the first error the device
 * scheduler reported since the last call (TILEQR_ERR_WATCHDOG), or a HIP
 * error; 0 if none. */
int qr_sync(void *stream);

/* Task trace of the last qr_factor launched with TILEQR_TRACE=1 in the
 * environment (development aid: shows where the DAG waits). Writes 9 int64
 * per task in ticket order (host, capacity cap tasks): type, i, j, k, strip,
 * ns when the task was taken, ns when its dependencies were met, ns when it
 * finished, workgroup id. *ntasks receives the count. Synchronizes. */
int qr_trace_fetch(int64_t *out, int64_t cap, int64_t *ntasks);

/* ---------------------------------------------------------------------- */
/* Single tile kernels (Section 2.1; used by the per-kernel checks)          */
/* ---------------------------------------------------------------------- */

/* Runs one task of the tile DAG of an M x N matrix with tiling (NB, IB),
 * all column strips, ignoring dependencies (the caller provides the inputs
 * the DAG would have produced):
 *   kind 0 GEQRT(k)         tile (k,k) -> R, V; T of tile (k,k)
 *   kind 1 TSQRT(i,k)       [R_kk; A_ik] -> R_kk, V_ik; T of tile (i,k)
 *   kind 2 LARFB(k,j)       A_kj <- Q_kk^T A_kj      (reads V_kk, T_kk)
 *   kind 3 SSRFB(i,j,k)     [A_kj; A_ij] <- Q_ik^T [A_kj; A_ij] (V_ik, T_ik)
 * Errors: -1 kind, -2 A, -3..-5 M, N, lda, -6 NB, -7 IB, -8 T, -9..-11 tile
 * indices out of range for the kind. */
int qr_tile_task(int kind, double *A, int64_t M, int64_t N, int64_t lda, int NB, int IB, double *T,
                 int i, int j, int k, void *stream);

/* Step 1 of the tuner (Section 5): kernel benchmark of DSSRFB. `workers`
 * workgroups (0 = one per compute unit) each apply `calls` full-tile DSSRFBs
 * (NB x NB tiles, inner block IB) to their own tiles, back to back, all timed
 * together (No Flush: tiles stay warm). *seconds (host) receives the elapsed
 * time of the whole launch. Errors: -1 NB, -2 IB, -3 calls, -4 workers,
 * -5 seconds null. */
int qr_ssrfb_bench(int NB, int IB, int calls, int workers, double *seconds);

/* Step 1 with cold caches (the flushed-cache timing of Section 5): the
 * same DSSRFB per workgroup as qr_ssrfb_bench, but each of the `calls`
 * calls in its own launch, preceded by a write over `flush_bytes` of scratch
 * device memory (0 = none) that evicts the tiles from the L2 caches and the
 * MALL; *seconds (host) sums the DSSRFB launches only. Errors: -1 NB, -2 IB,
 * -3 calls, -4 workers, -5 flush_bytes outside [0, 64 GiB], -6 seconds
 * null. */
int qr_ssrfb_bench_flush(int NB, int IB, int calls, int workers, int64_t flush_bytes,
                         double *seconds);

/* Measurement support (not an operation of the paper): the sustained rate
 * of v_mfma_f64_16x16x4f64, the FP64 matrix instruction of the DLARFB and
 * DSSRFB kernels, with register operands and eight independent accumulator
 * chains per wave, so that no memory access, barrier or dependence stall
 * limits it. wg_per_cu (1..8) workgroups of four waves run on every compute
 * unit, `iters` rounds of the eight products each. *tflops (host) receives
 * the whole chip's FP64 rate; *ghz (host, may be NULL) the shader clock the
 * probe measured over its own run. It is the ceiling that Step 1's rates
 * (Section 5) and the factorization's are read against, next to the published
 * peak. Errors: -1 wg_per_cu, -2 iters, -3 tflops null. */
int qr_mfma_probe(int wg_per_cu, int iters, double *tflops, double *ghz);

/* ---------------------------------------------------------------------- */
/* Tuning decision (Problem 2.1: instantaneous choice of (NB, IB))          */
/* ---------------------------------------------------------------------- */

/* Host only. Picks (NB, IB) for an M x N factorization in a batch of
 * `batch` matrices: TILEQR_NB / TILEQR_IB environment overrides first, then
 * the learned cost model if one is loaded and confident, then the decision
 * table's nearest benchmarked configuration (Section 6.1: nearest in
 * log M, log N, log batch; ties to the larger size) within the table section
 * tuned for the caller's compute units (the qr_set_compute_units setting,
 * else the whole device; the section whose budget is nearest in log scale,
 * as the paper interpolates over the core count), else the install
 * default (NB=128, IB=32, or the table's "default" line). *source: 0
 * default, 1 table, 2 model, 3 env;
 * +8 when the model was consulted but its ensemble spread exceeded 5 %
 * (the caller should run the pruned search for this shape). The spread is
 * the largest loss, against its own best candidate, that any model of the
 * ensemble predicts for the ensemble-mean choice. The model ranks flat-tree
 * pairs on the whole device, so it is not consulted where the table's entry
 * carries a row-domain count above 1 or belongs to a compute-unit budget.
 * Errors: -1 M < 0, -2 N < 0, -3 batch < 1, -4 NB null, -5 IB null. */
int qr_tune(int64_t M, int64_t N, int64_t batch, int *NB, int *IB, int *source);

/* Host only. The compute units the persistent grid of an M x N
 * factorization is sized for: the qr_set_compute_units setting if one is
 * made, else the decision table's nearest entry's units (0: all units).
 * qr_factor and qr_apply_Qt use this value. Errors: -1 M, -2 N, -3 batch,
 * -4 cus null. */
int qr_tune_units(int64_t M, int64_t N, int64_t batch, int *cus);

/* Host only. The row-domain count p of qr_factor_ca (p = 0 there) for an
 * M x N factorization: the decision table's nearest entry's (1 without a
 * table or when the entry has none). Errors: -1 M, -2 N, -3 batch, -4 p
 * null. */
int qr_tune_domains(int64_t M, int64_t N, int64_t batch, int *p);

/* Loads a decision table (host path; text: lines "entry M N batch NB IB
 * gflops [units [p]]", where units is the compute-unit count the grid is
 * sized for, 0 or absent for all, and p the row domains of qr_factor_ca
 * (absent: 1); lines "budget C" start a section of entries tuned for
 * callers limited to C compute units (0, the default: the whole device);
 * optional "default NB IB"; '#' comments), replacing the current one.
 * Returns 0, TILEQR_ERR_NOTABLE, or -1 for a null path. */
int qr_tune_load(const char *path);

/* Installs (or with nmodels = 0 removes) the ensemble of cost models used by
 * qr_tune. params (host): nmodels x 8769 floats (layout of qr_mlp_forward);
 * feat_mean/feat_std (host, 5 each) standardise the features, the model
 * predicts (log GFLOP/s - y_mean) / y_std; cand (host, 2*ncand ints) lists
 * the (NB, IB) candidates (each a valid tiling). Errors: -1 nmodels outside
 * [0, 64], -2 params null, -3 feat_mean null, -4 feat_std null or not
 * positive, -7 cand null, ncand outside [1, 4096] or an invalid pair. */
int qr_tune_set_model(const float *params, int nmodels, const float *feat_mean,
                      const float *feat_std, float y_mean, float y_std, const int *cand, int ncand);

/* ---------------------------------------------------------------------- */
/* Learned cost model: 5 -> 64 -> 64 -> 64 -> 1 MLP, ReLU, FP32             */
/* ---------------------------------------------------------------------- */
/* Parameter vector (8769 floats), weight matrices row-major [out][in]:
 *   W1[64][5] @0, b1[64] @320, W2[64][64] @384, b2[64] @4480,
 *   W3[64][64] @4544, b3[64] @8640, W4[1][64] @8704, b4[1] @8768.
 * Features per row (5 floats): log M, log N, log NB, IB/NB, batch count
 * (standardised by the caller). Loss: L = 1/(2n) sum (yhat - y)^2.
 * All pointers device, rows of X contiguous (n x 5 row-major). */

/* y[r] = model(X[r]) for `nmodels` models stored back to back in params;
 * y is nmodels x n (model-major). Errors: -1 params, -2 nmodels, -3 X,
 * -4 n, -5 y. */
int qr_mlp_forward(const float *params, int nmodels, const float *X, int64_t n, float *y,
                   void *stream);

/* Loss and full gradient of one model on a batch. grad: 8769 floats;
 * loss: 1 float (device). Errors: -1 params, -2 X, -3 y, -4 n, -5 grad,
 * -6 loss. */
int qr_mlp_grad(const float *params, const float *X, const float *y, int64_t n, float *grad,
                float *loss, void *stream);

/* Trains `nmodels` models at once (one workgroup each) with Adam
 * (beta1 0.9, beta2 0.999, eps 1e-8) on minibatches of `batch` rows drawn
 * by a counter-based generator from `seed` (model m uses seed + m).
 * params: nmodels x 8769 (in: initial weights, out: trained); adam: 2 x
 * nmodels x 8769 floats of optimizer state (zero it before the first call);
 * step0: Adam steps already taken (for bias correction when resuming);
 * loss_out: nmodels floats, mean training loss of the last epoch.
 * Errors: -1 params, -2 nmodels, -3 adam, -4 X, -5 y, -6 n, -7 epochs,
 * -8 batch, -9 lr, -11 loss_out. */
int qr_mlp_train(float *params, int nmodels, float *adam, const float *X, const float *y,
                 int64_t n, int epochs, int batch, float lr, uint64_t seed, int64_t step0,
                 float *loss_out, void *stream);

/* ---------------------------------------------------------------------- */
/* Host-only inspection of the tile DAG and its schedule                    */
/* ---------------------------------------------------------------------- */

/* Tile task counts (GEQRT, TSQRT, LARFB, SSRFB) of an M x N matrix with
 * tile order NB (strips not split). Errors: -1 M, -2 N, -3 NB, -4 counts. */
int qr_dag_counts(int64_t M, int64_t N, int NB, int64_t *counts);

/* Metric flops (Section 2.2): 4/3 N^3 for square, 2MN^2 - 2N^3/3 for
 * M >= N, 2NM^2 - 2M^3/3 for M < N. IB's extra flops are not counted. */
double qr_flops(int64_t M, int64_t N);

/* Flops the tile algorithm executes with inner blocking IB, counted task
 * by task (for the IB overhead of Section 2.2). */
double qr_flops_executed(int64_t M, int64_t N, int NB, int IB);

/* Builds the ticket order (as qr_factor_ca / qr_apply_Qt_ca would with p row
 * domains, for `workers` persistent workgroups; apply = 1 for the Q^T apply
 * with nrhs columns, 2 for the Q apply) and
 * checks it on the host: *seq = waits not yet satisfied when tasks run one
 * at a time in ticket order; *stress = data hazards (program-order
 * violations) seen in a randomised parallel replay with `workers` workers
 * (seed), or -1 if that replay deadlocked. Returns 0 or a positive error. */
int qr_plan_check(int64_t M, int64_t N, int NB, int IB, int p, int64_t nrhs, int apply,
                  int workers, uint64_t seed, int64_t *ntasks, int64_t *seq, int64_t *stress);

/* Writes the ticket order as 5 ints per task (type, i, j, k, strip) into
 * out (host, capacity cap tasks); *ntasks receives the count. Types: 0
 * GEQRT, 1 TSQRT, 2 LARFB, 3 SSRFB, 4 LARFB on B, 5 SSRFB on B, 6 TTQRT
 * (merge), 7 TTMQR (merge update), 8 TTMQR on B. */
int qr_plan_tasks(int64_t M, int64_t N, int NB, int IB, int p, int64_t nrhs, int apply,
                  int workers, int32_t *out, int64_t cap, int64_t *ntasks);

#ifdef __cplusplus
}
#endif

#endif /* TILEQR_H */
