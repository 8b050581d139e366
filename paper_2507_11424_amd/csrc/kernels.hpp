// Internal launch interface of the HIP kernels (host side).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace tnk {

// Compute modes of the contraction engine (mirrors tn_prec).
enum Prec : int { P_FP64 = 0, P_FP32 = 1, P_BF16X3 = 2, P_BF16X6 = 3 };

// A batched complex contraction written as a GEMM over gathered indices:
//   C[b](m, n) (+)= sum_k opA(A[b](m, k)) * opB(B[b](k, n))
// Element (m, k) of A lives at A + a_boff[b] + a_moff[m] + a_koff[k] (complex
// elements); likewise B and C.  opX conjugates when conjX is set.  The offset
// tables let one kernel contract tensors of any rank and index order without
// explicit transposes.
struct GettArgs {
    int M, N, K, batch;
    const void *A; const int32_t *a_moff; const int32_t *a_koff; const int64_t *a_boff;
    const void *B; const int32_t *b_koff; const int32_t *b_noff; const int64_t *b_boff;
    void *C; const int32_t *c_moff; const int32_t *c_noff; const int64_t *c_boff;
    int conjA, conjB;
    int accumulate;      // 1: C += product, 0: C = product
    int a_kfast;         // 1: A is contiguous along k (load lanes along k), 0: along m
    int b_kfast;         // 1: B is contiguous along k, 0: along n
    // split-K: ksplit slices of kchunk (multiple of 32) along k; slice z writes
    // its partial product to part[z][b][m][n] (dense, storage type) and a
    // reduction in fixed slice order writes C.  ksplit = 1: direct epilogue.
    int ksplit, kchunk;
    void *part;
    // k offsets: affine (offset of k = k * ks, no table read) or read from the
    // k table, which the kernel stages into LDS once (kchunk <= GETT_KTAB).
    int a_kaff, b_kaff;
    int a_ks, b_ks;
    // operand windows in bytes from each batch item's base (all offsets
    // reachable through the tables); operands are read with buffer loads whose
    // range check returns zero for padding, so a window must stay below 2^31.
    uint32_t a_bytes, b_bytes;
    // split-BF16 modes: A and B are packed bf16 planes (launch_pack_bf16) with
    // kpad columns (K rounded up to 32); a_bytes / b_bytes are one batch item's
    // planes
    int kpad;
    // optional tile skip: a tile whose item mask[coord / mask_div] equals
    // mask_skip is not computed (its part of C is left as it was); coord is the
    // batch index (mask_mode 1), the tile's first row m0 (2) or first column n0
    // (3).  For modes 2 and 3 mask_div must be a multiple of the tile edge
    // (else the launch ignores the mask).
    const int *mask;
    int mask_mode, mask_div, mask_skip;
};
// Largest K slice a block handles when a k table is not affine (LDS table).
constexpr int GETT_KTAB = 1024;
constexpr uint32_t GETT_MAX_WINDOW = 0x7FFFFFF0u;

// Tile configurations of the contraction kernel.
enum GettCfg : int {
    CFG_64x64 = 0,    // 4 waves, 32x32 per wave
    CFG_128x64 = 1,   // 4 waves, 64x32 per wave
    CFG_64x16 = 2,    // skinny N
    CFG_128x64W = 3,  // 8 waves, 32x32 per wave
    CFG_128x128W = 4, // 8 waves, 64x32 per wave (packed split-BF16 only)
    CFG_COUNT = 5
};

hipError_t launch_gett(const GettArgs &a, int prec, int cfg, hipStream_t s);
// Split-BF16 operand packing: element (row, k) of batch item b at
// X + boff[b] + roff[row] + (kaff ? k * ks : koff[k]) (complex64), conjugated if
// conj, split into np bf16 parts -> out[b][part][re/im][row][kpad] (zero past K).
hipError_t launch_pack_bf16(int np, const void *X, const int64_t *boff, const int32_t *roff, const int32_t *koff,
                            int kaff, int ks, int rows, int K, int kpad, int batch, int conj, void *out,
                            hipStream_t s);
void gett_tile(int cfg, int prec, int *bm, int *bn);

// ---------------------------------------------------------------- linear algebra
// Householder QR of `batch` complex matrices (m x n), FP64 arithmetic.
// Element (i, j) of matrix b of A: A + b*a_bs + i*a_rs + j*a_cs (complex
// elements of size esz: 16 = complex128, 8 = complex64), conjugated if a_conj.
// Outputs Q (m x k, k = min(m, n)) with the same addressing scheme, and R (k x n)
// if R != nullptr.  Workspace: see qr_workspace_bytes.
struct QrArgs {
    int m, n, batch;
    const void *A; int a_esz; int64_t a_bs, a_rs, a_cs; int a_conj;
    void *Q; int q_esz; int64_t q_bs, q_rs, q_cs; int q_conj;
    void *R; int r_esz; int64_t r_bs, r_rs, r_cs; int r_conj;
};
size_t qr_workspace_bytes(int m, int n, int batch);
hipError_t launch_qr(const QrArgs &a, void *workspace, hipStream_t s);
// Householder QR (one workgroup per matrix, global memory) of the batch items
// whose flags[b] has bit 4 set (a clamped Cholesky pivot), overwriting their Q
// (and R); the other items return at once.  The fallback of CholeskyQR for
// numerically rank-deficient input.  Its workspace holds at most 16 MiB of
// per-matrix slots (at least one): the workgroups loop over the batch.
size_t qr_fallback_workspace_bytes(int m, int n, int batch);
hipError_t launch_qr_fallback(const QrArgs &a, const int *flags, void *workspace, hipStream_t s);

// Cholesky of Hermitian G (batch x n x n, complex128, only the upper triangle is
// read) as G + shift * tr(G)/n * I = R^H R, Rinv = R^{-1} (upper triangular,
// complex128, batch x n x n) and, if Rf is not null, R itself.  A pivot below
// clamp * tr(G)/n is raised to it (flags[b] |= 4 when that happens).  One
// workgroup per matrix; n <= 64.
hipError_t launch_chol_inv(const double *G, int n, int batch, double shift, double clamp, double *Rinv, double *Rf,
                           int *flags, hipStream_t s);
// One CholeskyQR pass over row blocks of p.rb rows (see k_cqr_rows): rows of
// the batch x m x n (n <= 64) source, times the previous pass's inverse factor
// Ri when given, written to X (contiguous complex128) and/or dst (strided), and
// the partial Gram matrices of the blocks written to part
// ([batch][ceil(m / rb)][n][n], complex128) when given.
struct CqrPass {
    int m, n, batch, rb;
    const void *src; int s_esz; int64_t s_bs, s_rs, s_cs; int s_conj;
    const double *Ri;
    double *X;
    void *dst; int d_esz; int64_t d_bs, d_rs, d_cs; int d_conj;
    double *part;
};
int cqr_rows_per_block(int m);
// G[b] = sum over p of parts[b][p] (complex128, n x n each), in a fixed order.
hipError_t launch_sum_parts(const double *parts, int nparts, int n, int batch, double *G, hipStream_t s);
hipError_t launch_cqr_pass(const CqrPass &p, hipStream_t s);
// Batched SVD truncation (one-sided Jacobi, FP64): R [batch][n][n] complex128
// (row-major) = U diag(sigma) V^H with sigma descending; keeps the fewest k
// values whose discarded weight sum_{j>=k} sigma_j^2 is at most cutoff times
// the total, capped by the numerical rank (sigma > 1e-12 sigma_max), at least
// min(chi_min, rank).  Writes U[b](i, c) = u_c(i) and SV[b](c, l) = sigma_c
// conj(v_c(l)) for c < k, zero for c >= k (element size esz, 8 or 16), and
// kout[b] = k.  n <= SVD_NMAX; n > 64 needs svd_trunc_workspace_bytes.
// chi_max > 0 caps k; disc (optional, [batch]) receives the discarded weight
// sum_{j>=k} sigma_j^2 / sum_j sigma_j^2.
constexpr int SVD_NMAX = 256;
size_t svd_trunc_workspace_bytes(int n, int batch);
hipError_t launch_svd_trunc(const double *R, int n, int batch, double cutoff, int chi_min, void *U, void *SV, int esz,
                            int *kout, void *workspace, hipStream_t s, int chi_max = 0, double *disc = nullptr);
// From the SVD factors of Hermitian positive matrices M = U S V^H (the output
// of launch_svd_trunc: U and SV = S V^H, complex128, batch x n x n, n <= 64):
// Sq = U S^{1/2} V^H and Sp = U S^{-1/2} V^H over the kept values (zero rows of
// SV are dropped), the square root and its pseudo-inverse.
hipError_t launch_msg_roots(const double *U, const double *SV, int n, int batch, double *Sq, double *Sp,
                            hipStream_t s);
// U[:, c] *= sqrt(sigma_c), SV[c, :] /= sqrt(sigma_c) with sigma_c = |SV[c, :]|
// (complex128, batch x n x n, n <= 256): the balanced factors U S^{1/2}, S^{1/2} V^H.
hipError_t launch_split_sqrt(double *U, double *SV, int n, int batch, hipStream_t s);
// One entry of a block-copy table: a rows x cols block of complex128 elements
// read with row stride src_ld, written contiguously (row-major) at dst.
struct CopyBlock {
    const void *src;
    void *dst;
    int64_t rows, cols, src_ld;
};
// Runs the n entries of the DEVICE table tab (max_elems = the largest
// rows * cols, which sizes the grid).
hipError_t launch_copy_blocks(const CopyBlock *tab, int n, int64_t max_elems, hipStream_t s);
// x *= (re + i im) over n complex128 elements.
hipError_t launch_scale(void *x, int64_t n, double re, double im, hipStream_t s);
// out[b](i, j) = opA(in[b](i, j)) for an m x n matrix per batch item with element
// strides (bs, rs, cs) on both sides, element sizes ie / oe, conjugation if conj.
hipError_t launch_strided_copy(const void *in, int ie, int64_t ibs, int64_t irs, int64_t ics, void *out, int oe,
                               int64_t obs, int64_t ors, int64_t ocs, int m, int n, int batch, int conj,
                               hipStream_t s);

// ---------------------------------------------------------------- small kernels
// out[b] = sum |x[b][i]|^2 over n complex elements (FP64 accumulation), batch
// stride `bs`.  Deterministic two-level reduction; partial needs
// reduce_partial_count(n) * batch doubles.
int reduce_partial_count(int64_t n);
hipError_t launch_norm2(const void *x, int esz, int64_t n, int batch, int64_t bs,
                        double *partial, double *out, hipStream_t s);
// x[b] *= 1/sqrt(norm2[b]); logscale[b] (+)= 0.5 log(norm2[b]); flags[b] |= 1 if
// norm2 is not finite or not positive.
hipError_t launch_normalise(void *x, int esz, int64_t n, int batch, int64_t bs,
                            const double *norm2, double *logscale, int accumulate_log,
                            int *flags, hipStream_t s);
// Element-type conversion / copy (c128 <-> c64), n complex elements.
hipError_t launch_convert(const void *src, int src_esz, void *dst, int dst_esz, int64_t n,
                          hipStream_t s);
// Philox-uniform complex initial guess: element e of tensor gets counter
// (e, site, row, sample[b]) and key (seed, tag).
hipError_t launch_init_tensor(void *out, int esz, int64_t n, int batch, int64_t bs,
                              uint64_t seed, uint64_t tag, uint64_t row, uint64_t site,
                              const uint64_t *sample, hipStream_t s);
// batch n x n identity matrices, back to back.
hipError_t launch_eye(void *x, int esz, int n, int batch, hipStream_t s);
// Fill with a complex constant.
hipError_t launch_fill(void *x, int esz, int64_t n, double re, double im, hipStream_t s);
// out[b] = sum_i x[b][i] * y[b][i] (no conjugation), complex FP64 result (2 doubles).
// With a mask, items b with mask[b] == mask_skip are skipped (out[b] untouched).
hipError_t launch_dot(const void *x, const void *y, int esz, int64_t n, int batch, int64_t bs,
                      double *partial, double *out, hipStream_t s, const int *mask = nullptr, int mask_skip = 0);

// ---------------------------------------------------------------- sampler
struct DrawArgs {
    int batch;                 // samples in flight
    const double *pt0, *pt1;   // [batch][2]: complex P~(s) for s = 0 and s = 1
    const double *uniforms;    // [n_total][n_qubits] or nullptr
    int64_t u_row0;            // row of `uniforms` for batch entry 0
    int n_qubits, qubit;       // qubit drawn now
    uint64_t seed; const uint64_t *sample_index;  // Philox stream (when uniforms == nullptr)
    uint8_t *bits; int64_t bits_row0;              // bits [n_total][n_qubits]
    double *log_q;             // [batch]
    int *xsel;                 // [batch] out: drawn bit
    int *flags;                // [batch] |= 2 on a bad marginal
    double *log_cond;          // optional [n_total][n_qubits]: log P(x_q | earlier qubits)
};
hipError_t launch_draw(const DrawArgs &a, hipStream_t s);
// Gathers per-sample pointers: dst[b] = base_off + xsel[b] * stride.
hipError_t launch_select_offsets(const int *xsel, int batch, int64_t base_off, int64_t stride,
                                 int64_t *dst, hipStream_t s);
// out[b] = x[b][sel[b]] copy of a slab of n complex elements (slab stride ss).
hipError_t launch_select_copy(const void *x, int esz, int64_t n, int64_t ss, int64_t bs,
                              const int *sel, int batch, void *out, int64_t obs, hipStream_t s);
// out[b] = (sel[b] ? x1 : x0)[b], slabs of n complex elements, batch stride bs.
hipError_t launch_select2(const void *x0, const void *x1, int esz, int64_t n, int64_t bs, const int *sel,
                          int batch, void *out, hipStream_t s);
// Fill n doubles with v.
hipError_t launch_fill_f64(double *x, int64_t n, double v, hipStream_t s);
// Fill n ints with v.
hipError_t launch_fill_i32(int *x, int64_t n, int v, hipStream_t s);
// dots [4][2] = complex rho~[s][t] (order 00, 01, 10, 11) -> out[8] = rho / Tr rho.
hipError_t launch_env_rho(const double *dots, double *out, hipStream_t s);
// dots [4][2] = complex P~(s, t) -> p2[4] = Re P / sum Re P (if p2), zz = sum (-1)^(s+t) Re P / sum Re P.
hipError_t launch_env_p2(const double *dots, double *p2, double *zz, hipStream_t s);
// pt1[z] = exp(lnr[z]) tot[z] - pt0[z] (complex, [batch][2] doubles): the other
// projection's P~ from the traced total, whose right environment is stored
// divided by exp(lnr).  need[z] = 1 unless Re pt1[z] > thr * Re(exp(lnr) tot):
// a difference that small is left to a direct contraction.
hipError_t launch_marginal_rest(const double *tot, const double *lnr, const double *pt0, double *pt1, int batch,
                                double thr, int *need, hipStream_t s);
// out[z] = (xs[z] == other && !need[z]).
hipError_t launch_other_mask(const int *xs, const int *need, int other, int batch, int *out, hipStream_t s);
// For samples with xs[z] == other: log_q[z] += log(pd/(pf+pd)) - log(pu/(pf+pu)),
// pf = max(Re pt_f, 0), pu = max(Re pt_used, 0), pd = Re pt_direct (flags |= 2
// if pd is not positive and finite); log_cond (optional) gets log(pd/(pf+pd)).
hipError_t launch_fix_other(const double *pt_f, const double *pt_used, const double *pt_direct, const int *xs,
                            int other, int batch, double *log_q, double *log_cond, int64_t row0, int n_qubits,
                            int qubit, int *flags, hipStream_t s);
// Final amplitude -> log p.
// xs[z] = bits[(row0 + z) * n_qubits + qubit] (0/1) for z < batch.
hipError_t launch_bits_select(const uint8_t *bits, int64_t n_qubits, int64_t row0, int qubit, int batch, int *xs,
                              hipStream_t s);
// out[3] (device) = {log mean(p/q), mean(log q - log p + log_Z), effective sample
// size}; z_is[n_qubits] (optional) = importance-weighted <Z_q> from bits
// [n][n_qubits].  Three passes over stats_blocks(n) blocks with partial results
// in `workspace` (stats_workspace_bytes; every byte used is written before it is
// read, so it needs no clearing).
constexpr int STATS_BLOCKS_MAX = 64;
int stats_blocks(int64_t n);
size_t stats_workspace_bytes(int64_t n, int64_t n_qubits, bool with_z);
hipError_t launch_sample_stats(const double *log_q, const double *log_p, int64_t n, double log_Z,
                               const uint8_t *bits, int64_t n_qubits, double *out, double *z_is, void *workspace,
                               hipStream_t s);
// out[z * stride] = max_c k[c * batch + z] over c < cuts, or `constant` when
// k is null or cuts == 0.
hipError_t launch_chi_used(const int *k, int cuts, int batch, int constant, int *out, int64_t stride,
                           hipStream_t s);
// Content fingerprint of up to FP_MAX tensors: *acc += sum over tensors t and
// 8-byte words i of mix(word, salt[t] + i) (modulo 2^64; acc must be cleared by
// the caller).  A changed byte changes the sum except with probability ~2^-64.
constexpr int FP_MAX = 96;
struct FingerprintSet {
    int count;
    const void *ptr[FP_MAX];
    int64_t words[FP_MAX];
    uint64_t salt[FP_MAX];
};
hipError_t launch_fingerprint(const FingerprintSet &f, unsigned long long *acc, hipStream_t s);
hipError_t launch_logp(const double *amp, const double *mlog, int batch, double *log_p, double *arg,
                       hipStream_t s);

// ---------------------------------------------------------------- belief propagation
// out [4][N][Dm][Dm]: the message each site sends through each leg (0 up,
// 1 left, 2 down, 3 right); msg [N][4][Dm][Dm]: incoming messages; nbr [N][4]:
// the neighbour receiving through each leg, -1 without a bond.  Stores the
// Hermitian part of every sent message, normalised to unit Frobenius norm, as
// the neighbour's incoming message; dmax [N * 4] scratch; *delta = largest
// element change (infinity if a message vanished or overflowed).
hipError_t launch_bp_update(const void *out, void *msg, const int *nbr, int N, int Dm, double *dmax, double *delta,
                            hipStream_t s);
// outr [N][Dm][Dm]: the message each site would send to the right (pair closed
// with the other three messages).  out[0] = log|Z_BP|, out[1] = arg Z_BP with
// Z_BP = prod_v Z_v / prod_e Z_e; zv [N], ze [N][2] complex scratch.
hipError_t launch_bp_free_energy(const void *outr, const void *msg, const int *nbr, int N, int Dm, void *zv,
                                 void *ze, double *out, hipStream_t s);
// mats[q] (n x n complex128) <- pairs + off[q] (n x n), transposed if trans[q].
hipError_t launch_gather_mats(const void *pairs, const int64_t *off, const int *trans, int count, int n, void *mats,
                              hipStream_t s);
// Eigenvalues of `batch` general complex n x n matrices (overwritten), one
// lane each: Householder Hessenberg reduction and shifted QR with deflation.
// lam [batch][n] complex128; eps[q] = 1 - max|lambda| / sum|lambda|; info[q] = 1
// if the iteration limit was reached.
constexpr int BP_EIG_NMAX = 256;
hipError_t launch_eig(void *mats, int n, int batch, void *lam, double *eps, int *info, hipStream_t s);

}  // namespace tnk
