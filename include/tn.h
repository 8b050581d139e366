/*
 * tn.h -- C ABI of the MI355X boundary-MPS contraction and sampling library.
 *
 * The operations follow Rudolph & Tindall, "Simulating and Sampling from
 * Quantum Circuits with 2D Tensor Networks":
 *
 *   tn_boundary_contract  norm <psi|psi> of a planar tensor-network state by
 *                         boundary MPSs passed through its rows in reverse
 *                         order, each MPS-MPO product compressed to bond chi by
 *                         one-site variational fitting (Methods, "The Boundary
 *                         Matrix Product State Method"; Appendix, "Sampling
 *                         from a Tensor Network State", Fig. 7c-d).  The stored
 *                         boundary set is kept in the handle for sampling.
 *   tn_environments       one-site density matrices and nearest-neighbour
 *                         <ZZ> by direct boundary-MPS contraction (Results,
 *                         Fig. 4, "direct contraction").
 *   tn_sample             sequential bitstring sampling, row by row and qubit
 *                         by qubit from one-site reduced density matrices
 *                         conditioned on the amplitude boundary above and the
 *                         stored norm boundary below; q(x) is the product of
 *                         the conditionals and p(x) comes from the last
 *                         amplitude boundary (Appendix, sampling; Fig. 7d).
 *
 * Conventions for every call:
 *  - Device pointers are HIP device memory on the handle's device; host
 *    pointers are ordinary host memory.  The caller owns every input and output
 *    buffer; the library owns only its workspace and the cached boundary set.
 *  - Work is enqueued on the handle's stream.  Calls that return host scalars
 *    synchronise that stream; the others are asynchronous.
 *  - Errors are returned as tn_status; no exception crosses the ABI.  On error
 *    the outputs are unspecified and tn_last_error() describes the failure.
 *  - One handle must not be used by two threads at once.
 *  - The cached norm boundary set: tn_boundary_contract (direction 0) always
 *    recomputes it; tn_environments and tn_sample reuse it only when the
 *    lattice, the options chi, sweeps, init, prec and init_seed, the site
 *    pointers and a 64-bit fingerprint of the site tensors' bytes (computed on
 *    the device at every call) all equal those of the call that computed it,
 *    and recompute it otherwise.  A state overwritten in place, or a new state
 *    placed at an old one's addresses, therefore gets a fresh set.
 *
 * Site tensor layout: complex, interleaved (re, im), row-major with index order
 * [p][u][l][d][r] (physical, up, left, down, right).  A bond that is absent or
 * leaves the grid has dimension 1; a grid position without a qubit has p = 1:
 * a dummy (every bond 1, the tensor is a scalar) or a tensor without a
 * physical index that carries bonds, such as the junction of a staggered-row
 * partition that splits a fused pair of diagonal bonds into its left and right
 * legs.
 */
#ifndef TN_H
#define TN_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct tn_handle tn_handle;

typedef enum {
    TN_OK = 0,
    TN_ERR_INVALID = 1,     /* null pointer, bad enum, bad option value          */
    TN_ERR_SHAPE = 2,       /* inconsistent lattice dimensions                   */
    TN_ERR_OOM = 3,         /* device allocation failed or workspace cap reached */
    TN_ERR_HIP = 4,         /* a HIP runtime call failed (incl. no device)       */
    TN_ERR_NUMERIC = 5,     /* non-finite or non-positive norm or marginal       */
    TN_ERR_UNSUPPORTED = 6  /* valid request outside what this library implements */
} tn_status;

typedef enum { TN_C128 = 0, TN_C64 = 1 } tn_dtype;

/* Arithmetic of the bulk contractions.  QR, norms, renormalisation and the
 * probability normalisation are FP64 in every mode. */
typedef enum {
    TN_PREC_FP64 = 0,    /* complex128 storage, FP64 MFMA                           */
    TN_PREC_FP32 = 1,    /* complex64 storage, FP32 MFMA                            */
    TN_PREC_BF16X3 = 2,  /* complex64 storage, each FP32 operand split into two BF16
                            parts (hi + lo), three BF16 MFMA products, FP32 accumulate */
    TN_PREC_BF16X6 = 3   /* as BF16X3 with three parts and six products             */
} tn_prec;

/* A planar tensor-network state embedded in a rows x cols grid; partitions are
 * the rows (Methods: partitions forming a line). */
typedef struct {
    int32_t rows, cols;
    const int32_t *phys;        /* host [rows*cols]: 2 for a qubit, 1 for a non-qubit    */
    const int32_t *dim_h;       /* host [rows*(cols-1)]: bond (r,c)-(r,c+1), >= 1        */
    const int32_t *dim_v;       /* host [(rows-1)*cols]: bond (r,c)-(r+1,c), >= 1        */
    const int32_t *site_index;  /* host [rows*cols]: bit position of the qubit, -1 else  */
    tn_dtype dtype;             /* element type of every site tensor                     */
    const void *const *site;    /* host array [rows*cols] of DEVICE pointers, layout above */
} tn_peps;

typedef struct {
    int32_t chi;          /* max bond of the norm boundary MPS (paper: R_n)            */
    int32_t chi_x;        /* max bond of the sampler's amplitude boundary (paper: R_x)  */
    int32_t sweeps;       /* full one-site fit sweeps per MPS-MPO product (>= 1)        */
    int32_t direction;    /* norm only: 0 bottom-up (rows last to first), 1 top-down,
                             2 / 3 the same over columns.  Environments and sampling
                             use rows, bottom-up boundaries (paper's order).           */
    int32_t init;         /* 0: exact product + QR canonicalisation when chi reaches the
                             exact bound, else fit from a random guess; 1: always fit    */
    tn_prec prec;
    uint64_t init_seed;   /* Philox key of the random initial guesses                  */
    size_t workspace_cap; /* bytes of device workspace the library may hold; 0 = no cap */
    double svd_cutoff;    /* sampler only: > 0 truncates every fitted amplitude boundary
                             by an SVD sweep keeping, per cut, the fewest singular values
                             whose discarded weight sum_{j>=k} s_j^2 / sum_j s_j^2 is
                             <= svd_cutoff (the error measure of Eq. error_per_gate);
                             0 = fixed bond chi_x (the paper's sampler)                 */
    int32_t chi_x_min;    /* lower clamp of that truncation (never above the numerical
                             rank, s_j > 1e-12 s_0); the upper clamp is chi_x <= 256    */
} tn_opts;

/* Fills opts with defaults: chi = chi_x = 16, sweeps = 2, direction 0, init 0,
 * FP64, seed 0, no cap, svd_cutoff 0, chi_x_min 1. */
void tn_default_opts(tn_opts *opts);

/* Creates a handle bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t, NULL = the null stream).  TN_ERR_HIP if the device is absent. */
tn_status tn_create(tn_handle **h, int device, void *hip_stream);

/* Frees the handle, its workspace and cached boundary set (synchronises). */
tn_status tn_destroy(tn_handle *h);

/* Norm Z = <psi|psi> by boundary MPS (see top of file).  Writes log|Z| and
 * arg Z to host doubles.  Caches the bottom-up boundary set when direction is 0.
 * Synchronises the stream. */
tn_status tn_boundary_contract(tn_handle *h, const tn_peps *peps, const tn_opts *opts,
                               double *log_abs_Z, double *arg_Z);

/* One-site density matrices and nearest-neighbour <ZZ> from the boundary MPSs
 * above and below every row (two-row environments for vertical pairs).
 *   rho1 : device [rows*cols][2][2] complex128 (8 doubles per site), rho / Tr rho,
 *          NaN for dummy sites;
 *   zz_h : optional (NULL) device [rows*(cols-1)] doubles, <Z Z> of (r,c),(r,c+1),
 *          NaN if either site is a dummy;
 *   zz_v : optional (NULL) device [(rows-1)*cols] doubles, same for (r,c),(r+1,c);
 *   p2_h, p2_v : optional (NULL) device [bonds][4]: diagonal of the normalised
 *          two-site marginal in the order 00, 01, 10, 11.
 * Horizontal (vertical) pairs are contracted only if zz_h or p2_h (zz_v or p2_v)
 * is given.  Synchronises the stream. */
tn_status tn_environments(tn_handle *h, const tn_peps *peps, const tn_opts *opts,
                          double *rho1, double *zz_h, double *zz_v,
                          double *p2_h, double *p2_v);

/* Draws samples first_sample .. first_sample+n-1 (paper's sampler).  Samples
 * run in waves sized to the free device memory; the launch sequence of the
 * second full wave is captured into a HIP graph and replayed for the later
 * full waves of the call (same kernels, arguments and memory, so the results
 * equal those of running every wave directly); with timing enabled
 * (tn_set_timing) every wave runs directly, so that each launch is timed.
 *   uniforms : optional device [n][N] doubles in [0,1) (N = number of qubits):
 *              the uniform that draws qubit q of sample i; NULL = Philox4x64-10
 *              with key (seed, 3) and counter (q, first_sample+i, 0, 0), the
 *              uniform being (word0 >> 11) * 2^-53;
 *   bits     : device [n][N] uint8, bit of qubit q at position site_index;
 *   log_q    : device [n] doubles, log of the product of drawn conditionals;
 *   log_p    : optional device [n] doubles, 2 log|<x|psi>| from the last
 *              amplitude boundary (accurate only when chi_x is large);
 *   chi_x_used : optional device [n][rows] int32, the largest bond kept by the
 *              amplitude boundary that conditions each row (1 for the first
 *              row; with svd_cutoff > 0 it varies per sample).
 * Computes (and caches) the norm boundary set if the cached one does not match
 * the state and options (rule at the top of this file).  A sample is a function of (state, options, seed,
 * sample index) only, so split runs reproduce one run.
 * Synchronises the stream (marginal checks). */
tn_status tn_sample(tn_handle *h, const tn_peps *peps, const tn_opts *opts,
                    uint64_t seed, uint64_t first_sample, int64_t n,
                    const double *uniforms, uint8_t *bits, double *log_q, double *log_p,
                    int32_t *chi_x_used);

/* Independent check of given bitstrings (Methods, sampling paragraphs: p(x)
 * recomputed by a separate contraction of <x|psi> rather than taken from the
 * sampler).  The single-layer network <x|psi> is contracted row by row, top
 * down, with boundary MPSs of bond <= opts->chi_x fitted by the one-site fit
 * (the paper uses twice the PEPS bond dimension for this check); the initial
 * guesses use Philox4x64-10 key (init_seed, 4) with the sample index
 * first_sample + i in the counter, a stream disjoint from the sampler's.
 *   bits  : device [n][N] uint8 (0/1, qubit q at column site_index), read only;
 *   log_p : device [n] doubles, 2 log|<x|psi>| (-inf for a zero amplitude);
 *   arg   : optional device [n] doubles, arg <x|psi> in (-pi, pi].
 * Independent of the cached boundary set; asynchronous on the handle's stream. */
tn_status tn_amplitude(tn_handle *h, const tn_peps *peps, const tn_opts *opts,
                       uint64_t first_sample, int64_t n, const uint8_t *bits,
                       double *log_p, double *arg);

/* Belief propagation (BP) on the norm network <psi|psi> and the loop BP error
 * (Methods, "Quantum Circuit Simulation": message tensors from BP, exact
 * without loops; "The Boundary Matrix Product State Method": BP contraction
 * and Eqs. avBPError, loopBPerror; Appendix, "Applying Gates to a Tensor
 * Network State": message update and normalisation; "Computing the BP Error").
 * Messages live on every bond in both directions as D x D matrices over the
 * bond's ket and bra indices; they start as identity / sqrt(D) and are updated
 * in parallel sweeps: the message a site sends through a bond is the site's
 * (A, conj A) pair closed with its incoming messages on its other bonds, taken
 * as its Hermitian part (exact arithmetic keeps it Hermitian; rounding would
 * otherwise seed the update's unstable anti-Hermitian directions) and divided
 * by its Frobenius norm.  Sweeps stop when the largest element change is below
 * tol (checked every 4 sweeps) or after max_sweeps.  FP64 throughout; the
 * state may be complex128 or complex64.
 *   log_abs_Z, arg_Z : host, Z_BP = prod_sites Z_v / prod_bonds Z_e (Z_v the
 *                      pair closed with all its messages, Z_e = sum m_{v->w}
 *                      m_{w->v} elementwise);
 *   sweeps, last_change : optional host outputs;
 *   eps_mean, eps_loops, n_loops : optional host outputs of the loop BP error;
 *                      the primitive loops are the bounded faces of the grid
 *                      embedding (grid cells merged across absent bonds),
 *                      ordered by their first site (row-major); eps_l = 1 -
 *                      |lambda_1| / sum |lambda_i| over the eigenvalues of the
 *                      loop's transfer matrix (BP messages on the loop's
 *                      boundary, one loop bond cut open); eps_loops holds
 *                      eps_capacity entries (TN_ERR_INVALID if there are more
 *                      loops; n_loops is written first).  Bond dimensions up to
 *                      16 (transfer matrices up to 256 x 256).
 *   messages         : optional DEVICE buffer [rows*cols][4][Dm][Dm] complex128
 *                      (Dm = the largest bond; legs up, left, down, right;
 *                      message into the site; padded entries zero; legs
 *                      without a bond hold e0 e0^T).
 * Synchronises the stream.  TN_ERR_NUMERIC if a message vanishes or the
 * eigenvalue iteration does not converge. */
tn_status tn_bp(tn_handle *h, const tn_peps *peps, int max_sweeps, double tol, double *log_abs_Z, double *arg_Z,
                int *sweeps, double *last_change, double *eps_mean, double *eps_loops, int eps_capacity,
                int *n_loops, void *messages);

/* Circuit simulation by BP-gauged simple update (Methods, "Quantum Circuit
 * Simulation", Eqs. error_per_gate and total_fidelity; Appendix, "Applying
 * Gates to a Tensor Network State").  Applies n_gates two-qubit gates, in list
 * order, to the state `peps` and writes the result to site_out (host array
 * [rows*cols] of DEVICE pointers, each sized and typed like the matching input
 * site; it may equal the input's to update in place).  Bond dimensions stay
 * those of the lattice.
 *   gate_sites  host [n_gates][5] int32: group, r, c, r2, c2 with (r2, c2) =
 *               (r, c+1) or (r+1, c), both sites qubits.  The BP messages of
 *               the norm network are recomputed whenever `group` differs from
 *               the previous gate's.  Gates of one group must share no qubit
 *               (TN_ERR_INVALID otherwise): they see the same messages
 *               and are applied together, batched by orientation and
 *               site shapes.
 *   gates       host complex128 4 x 4 row-major unitaries in the basis 2a + b,
 *               a the qubit at (r, c): gate_stride 16 = one matrix per gate,
 *               0 = one matrix for all.
 *   bp_max_sweeps, bp_tol  BP schedule (as tn_bp).
 *   eps         host [n_gates] out: the discarded weight of each gate's
 *               normalised singular values, sum_{j>=D} s_j^2 / sum_j s_j^2.
 *   fidelity    host out (may be NULL): prod_i (1 - eps_i).
 *   messages_in   optional DEVICE [rows*cols][4][Dm][Dm] complex128 (the
 *                 layout of tn_bp's messages, Dm = the largest bond): the
 *                 first group's BP starts from them instead of identity /
 *                 sqrt(D) -- pass an earlier call's messages_out to continue
 *                 a circuit split over several calls exactly as one call.
 *   messages_out  optional DEVICE, same layout (may equal messages_in): the
 *                 last group's converged messages.
 * Per gate: the pair gauged with the square roots of its incoming messages
 * (pseudo-inverse roots to undo it; message eigenvalues at or below 1e-12 of
 * the largest taken as 0), reduced by QR, the gate applied, an SVD kept to
 * min(D, rank) values (rank: above 1e-12 of the largest) split as U S^1/2 and
 * S^1/2 V^H.  FP64 arithmetic whatever the input type (complex64 results are
 * rounded once on output).  Bonds up to 64 (pair matrices up to 256 wide).
 * Synchronises the stream.
 * TN_ERR_INVALID for a malformed gate list, TN_ERR_UNSUPPORTED above the bond
 * limit. */
tn_status tn_simple_update(tn_handle *h, const tn_peps *peps, void *const *site_out, int n_gates,
                           const int32_t *gate_sites, const double *gates, int gate_stride, int bp_max_sweeps,
                           double bp_tol, double *eps, double *fidelity, const void *messages_in,
                           void *messages_out);

/* Sample-quality metrics from per-sample log q and log p (device [n] doubles,
 * natural logs), with w_i = p(x_i)/q(x_i) (Methods, the unbiased norm
 * estimator, Eq. kld and the importance-sampling formula, read in its
 * self-normalised form):
 *   out[0] = log((1/n) sum_i w_i), the estimate of log <psi|psi>;
 *   out[1] = (1/n) sum_i (log q_i - log p_i + log_Z), the sample KLD against
 *            p / Z with log_Z from tn_boundary_contract;
 *   out[2] = (sum w)^2 / sum w^2, the effective sample size;
 * out is host memory (3 doubles).  z_is (optional device [n_qubits] doubles)
 * receives sum_i w_i (1 - 2 x_iq) / sum_i w_i, which needs bits (device
 * [n][n_qubits] uint8).  n must be > 0.  Synchronises the stream. */
tn_status tn_sample_stats(tn_handle *h, int64_t n, int32_t n_qubits, const uint8_t *bits,
                          const double *log_q, const double *log_p, double log_Z,
                          double *out, double *z_is);

/* Allocation-free variant of tn_sample_stats, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same inputs and metrics, computed by the same
 * kernels, but:
 *   out  : DEVICE [3] doubles (not host memory); the call is asynchronous on
 *          the handle's stream and never synchronises;
 *   the partial results live in a fixed scratch array of 4 MiB per device,
 *   held until the process ends: with z_is it holds up to
 *   TN_NOALLOC_MAX_QUBITS qubits (any n); more qubits are rejected with
 *   TN_ERR_INVALID before anything is launched.
 * The call performs no device allocation or free.  All calls on one device
 * share that scratch: calls that overlap on one device (two streams, or two
 * threads) race and must be serialised by the caller.  Errors as
 * tn_sample_stats. */
#define TN_NOALLOC_MAX_QUBITS 8188
tn_status tn_sample_stats_noalloc(tn_handle *h, int64_t n, int32_t n_qubits, const uint8_t *bits,
                                  const double *log_q, const double *log_p, double log_Z, double *out, double *z_is);

/* Text of the last error on this handle ("" if none).  Valid until the next call. */
const char *tn_last_error(const tn_handle *h);

/* Work counters of the last call: the flops of every contraction kernel
 * launch (8 real flops per complex multiply-add, summed over the actual index
 * dimensions), the launch count, and -- when timing is enabled -- the summed
 * device time of those launches and of the QR / orthonormalisation calls in
 * milliseconds (HIP events on the handle's stream).  The orthonormalisation
 * issues contractions of its own (Gram matrices, triangular solves): they are
 * included in gemm_* and in qr_ms, and their flops are also reported in
 * qr_gemm_flops, so gemm_flops - qr_gemm_flops is the method's own work.
 * The sampler extends the environment of the rarer outcome only for the
 * samples that drew it: those launches skip the other samples' tiles, and are
 * counted apart (masked_launches, masked_ms), outside gemm_*.  gemm_bytes:
 * algorithmic operand bytes of the counted launches (A and B read once, C
 * written once, and read once more when accumulating).  graph_launches: the
 * sampler waves replayed from a captured launch graph (their contraction
 * launches are included in the other counters).
 * Any pointer may be NULL. */
tn_status tn_get_counters(const tn_handle *h, double *gemm_flops, int64_t *gemm_launches,
                          double *gemm_ms, double *qr_ms, int64_t *qr_launches,
                          double *qr_gemm_flops, int64_t *masked_launches, double *masked_ms,
                          double *gemm_bytes, int64_t *graph_launches);

/* Enables (1) or disables (0) per-launch HIP-event timing: an event pair is
 * recorded around every contraction and QR launch on the handle's stream and read
 * when a call returns (no waits between launches). */
tn_status tn_set_timing(tn_handle *h, int enable);

/* Enables (1) or disables (0) autotuning of the contraction kernels.  When on,
 * the first call of each contraction shape that overwrites its output times
 * every tile configuration and split-K choice of the GETT kernel on that call's
 * operands (waiting for the stream) and keeps the fastest for the handle's
 * lifetime; results differ from the untuned choice only in the rounding of the
 * K summation order.  cache_path (host string, may be NULL) names a text file
 * whose choices are loaded now and to which new choices are appended; a missing
 * file is not an error.  Errors: TN_ERR_INVALID for a NULL handle. */
tn_status tn_set_autotune(tn_handle *h, int enable, const char *cache_path);

/* Writes into buf (host, len bytes, NUL-terminated, truncated if short) a
 * tab-separated table of the `top` contraction shapes with the most device time
 * recorded in timing mode since the handle was created: milliseconds, calls,
 * TFLOP/s and the shape (letters, M, N, K, batch, tile, split). */
tn_status tn_plan_report(const tn_handle *h, int top, char *buf, size_t len);

/* ---------------------------------------------------------------------------
 * Kernel test hooks: run one engine primitive on caller buffers so that its
 * numerics can be checked in isolation.  Not needed by applications.
 *
 * tn_test_contract: C[ic] (+)= sum A[ia] * B[ib] (einsum letters, one char per
 *   index, row-major dense DEVICE tensors of the precision's storage type:
 *   complex128 for FP64, complex64 otherwise); dims are host arrays of
 *   strlen(letters) entries; conjA/conjB conjugate an operand; accumulate adds;
 *   cfg >= 0 forces a tile configuration (0: 64x64, 1: 128x64, 2: 64x16,
 *   3: 128x64 on 8 waves) and ksplit > 0 a number of K slices, -1 / 0 = the
 *   planner's choice.  Enqueued on the handle's stream.
 * tn_test_qr: reduced QR (FP64 arithmetic) of `batch` row-major m x n DEVICE
 *   matrices of element size esz (16 or 8 bytes): Q is m x k, R (optional,
 *   NULL = not formed) is k x n, k = min(m, n).  method 0: Householder;
 *   method 1: the fit's shifted CholeskyQR3 (m >= n, n <= 64; Householder
 *   otherwise), R = R_3 R_2 R_1.  method 2: CholeskyQR3 of the LQ moves, Q
 *   only (R must be NULL, m >= n): A and Q hold the conjugate transposes
 *   (n x m, row-major), so the rows of Q are an orthonormal basis of the rows
 *   of A.  Enqueued on the handle's stream.
 * tn_test_svd: the sampler's SVD truncation step on `batch` row-major n x n
 *   complex128 DEVICE matrices R (n <= 256): U (n x n) and SV (n x n), element
 *   size esz (16 or 8), with R ~ U SV; columns of U and rows of SV past the
 *   kept count are zero; k (device int32 [batch]) receives the kept counts
 *   (rule as for tn_opts.svd_cutoff with the lower clamp chi_min).  Enqueued
 *   on the handle's stream.
 */
tn_status tn_test_contract(tn_handle *h, int prec, const char *ia, const void *A, const int32_t *adims,
                           int conjA, const char *ib, const void *B, const int32_t *bdims, int conjB,
                           const char *ic, void *C, const int32_t *cdims, int accumulate,
                           int cfg, int ksplit);
tn_status tn_test_qr(tn_handle *h, int m, int n, int batch, int esz, const void *A, void *Q, void *R,
                     int method);
tn_status tn_test_svd(tn_handle *h, int n, int batch, const void *R, double cutoff, int chi_min, void *U, void *SV,
                      int esz, int32_t *k);
/* tn_test_set_mask: later tn_test_contract calls skip the output tiles of the
 *   items i of index letter `letter` with mask[i] == 0 (device int32 array
 *   over that letter's extent; those parts of C keep their contents), as the
 *   sampler's s = 1 environment steps do; mask = NULL clears it.  The skip
 *   applies when the letter is the slowest of the contraction's batch, row or
 *   column indices and its blocks align with the tiles, else everything is
 *   computed. */
tn_status tn_test_set_mask(tn_handle *h, const int32_t *mask, char letter);
/* tn_test_eig: eigenvalues of `batch` general complex n x n DEVICE matrices A
 *   (complex128, row-major, read only; n <= 256) by the kernel of tn_bp's loop
 *   error: lam (device [batch][n] complex128, unordered), eps (device [batch]
 *   doubles: 1 - max|lambda| / sum|lambda|), info (device [batch] int32, 1 if
 *   the iteration limit was reached).  Enqueued on the handle's stream. */
tn_status tn_test_eig(tn_handle *h, int n, int batch, const void *A, void *lam, double *eps, int32_t *info);
/* tn_test_sample_config: later tn_sample calls on this handle run waves of
 *   `wave` samples (0 = sized from free device memory), stop after the first
 *   `rows_limit` rows (0 = all; bits of later rows are 0, log_q is the partial
 *   sum, log_p is NaN), and, if log_cond is not NULL, write into it (device
 *   [n][N] doubles, same indexing as bits) log P(x_q | earlier qubits) for
 *   every drawn qubit q (entries of undrawn qubits are left as they were).
 *   graphs = 1 (the default) replays the full waves after the second from the
 *   captured launch graph of the second; 0 runs every wave directly.
 *   Calling it with (0, 0, NULL, 1) restores the defaults.  Errors:
 *   TN_ERR_INVALID for a NULL handle, negative wave / rows_limit or graphs
 *   other than 0 and 1. */
tn_status tn_test_sample_config(tn_handle *h, int wave, int rows_limit, double *log_cond, int graphs);

#ifdef __cplusplus
}
#endif

#endif /* TN_H */
