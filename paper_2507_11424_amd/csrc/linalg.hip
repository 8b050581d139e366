// FP64 linear algebra of the boundary-MPS fit: Householder QR of the tall
// (chi * phys) x chi site matrices (the gauge moves of the one-site fit), norms,
// renormalisation, Philox initial guesses.
//
// QR is a tall-skinny (TSQR) tree: the rows are split into balanced blocks of at
// most QR_LDS / n rows, each block is factored by one workgroup entirely in LDS
// (Householder, wavefront reductions), the stacked n x n R factors are factored
// the same way level by level, and the explicit thin Q is formed top-down by
// applying each block's reflectors to its chunk of the parent Q.  Matrices with
// more than 64 columns that do not fit one block fall back to a one-workgroup
// factorisation in global memory.
#include "kernels.hpp"

#include <algorithm>
#include <cmath>
#include <vector>

namespace tnk {
namespace {

constexpr int QR_NT = 256;
constexpr int CQR_ROWS = 32;  // rows of a CholeskyQR pass staged in LDS at a time
constexpr int CQR_LD = 65;    // padded LDS row of those passes (complex doubles)
constexpr int SUM_E = 8;      // entries per workgroup of the partial-sum reduction
constexpr int QR_LDS = 8192;  // complex doubles held by one workgroup (128 KiB)
constexpr int QR_G = QR_NT / 64;

struct MatDesc {
    const void *p; int esz; int64_t bs, rs, cs; int conj;
};
struct MatOut {
    void *p; int esz; int64_t bs, rs, cs; int conj;
};

__device__ inline double2 ld_c(const void *base, int esz, int64_t off, int conj) {
    double2 v;
    if (esz == 16) {
        v = reinterpret_cast<const double2 *>(base)[off];
    } else {
        const float2 f = reinterpret_cast<const float2 *>(base)[off];
        v.x = f.x; v.y = f.y;
    }
    if (conj) v.y = -v.y;
    return v;
}
__device__ inline void st_c(void *base, int esz, int64_t off, double2 v, int conj) {
    if (conj) v.y = -v.y;
    if (esz == 16) {
        reinterpret_cast<double2 *>(base)[off] = v;
    } else {
        reinterpret_cast<float2 *>(base)[off] = make_float2((float)v.x, (float)v.y);
    }
}
__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cmulc(double2 a, double2 b) {  // conj(a) * b
    return make_double2(a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x);
}

__device__ inline double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
// Block sum over QR_NT threads; every thread receives the result.
__device__ inline double block_sum(double v, double *red) {
    v = wave_sum(v);
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < QR_NT / 64; ++i) s += red[i];
    return s;
}

// Block maximum over QR_NT threads; every thread receives the result.
__device__ inline double block_max(double v, double *red) {
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    const int w = threadIdx.x >> 6;
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[w] = v;
    __syncthreads();
    double m = 0.0;
#pragma unroll
    for (int i = 0; i < QR_NT / 64; ++i) m = fmax(m, red[i]);
    return m;
}

// Below this sum of squares a column's norm is recomputed from values scaled
// by its largest modulus: squares of entries under ~1e-154 fall into the
// subnormal range (or to zero) and would give an inaccurate norm.
constexpr double HH_SMALL2 = 1e-280;

// In-place Householder factorisation of X (rows x n, leading dimension ld).
// After return: X[i][j], i >= j, holds reflector j normalised to v_j[0] = 1
// (the 1 stored on the diagonal); X[i][j], i < j, holds R; beta[j] = R[j][j];
// tau[j] = 2 / ||v_j||^2 = (|alpha| + sigma) / sigma, between 1 and 2 (0 for a
// zero column).  H_j = I - tau_j v_j v_j^H is Hermitian and unitary; A = H_0 ...
// H_{k-1} R.  With the normalised reflector nothing in the step scales like
// 1 / sigma^2, so columns whose remaining norm is far below the others' (the
// rank-deficient matrices of gauged site tensors) stay finite and exact.
__device__ void hh_factor(double2 *X, int rows, int n, int ld, double2 *beta, double *tau,
                          double *red, double2 *wpart) {
    const int t = threadIdx.x;
    const int kmax = rows < n ? rows : n;
    for (int j = 0; j < kmax; ++j) {
        double s = 0.0;
        for (int i = j + t; i < rows; i += QR_NT) {
            const double2 x = X[(int64_t)i * ld + j];
            s += x.x * x.x + x.y * x.y;
        }
        s = block_sum(s, red);
        double sigma = sqrt(s);
        if (s < HH_SMALL2) {  // uniform over the block
            double cm = 0.0;
            for (int i = j + t; i < rows; i += QR_NT) {
                const double2 x = X[(int64_t)i * ld + j];
                cm = fmax(cm, fmax(fabs(x.x), fabs(x.y)));
            }
            cm = block_max(cm, red);
            double s2 = 0.0;
            if (cm > 0.0) {
                for (int i = j + t; i < rows; i += QR_NT) {
                    const double2 x = X[(int64_t)i * ld + j];
                    const double xr = x.x / cm, xi = x.y / cm;
                    s2 += xr * xr + xi * xi;
                }
            }
            s2 = block_sum(s2, red);
            sigma = cm > 0.0 ? cm * sqrt(s2) : 0.0;
        }
        const double2 alpha = X[(int64_t)j * ld + j];
        const double aabs = hypot(alpha.x, alpha.y);
        __syncthreads();
        double tj = 0.0;
        double2 bj = make_double2(0.0, 0.0);
        if (sigma > 0.0) {
            const double2 ph = aabs > 0.0 ? make_double2(alpha.x / aabs, alpha.y / aabs) : make_double2(1.0, 0.0);
            const double d = aabs + sigma;  // |v_j[0]| before normalisation
            bj = make_double2(-ph.x * sigma, -ph.y * sigma);
            tj = d / sigma;
            // v_j[i] = x_i / (ph d) below the diagonal (divisions, not a
            // reciprocal: d may be subnormal)
            for (int i = j + 1 + t; i < rows; i += QR_NT) {
                const double2 x = X[(int64_t)i * ld + j];
                const double2 xc = cmulc(ph, x);  // conj(ph) x
                X[(int64_t)i * ld + j] = make_double2(xc.x / d, xc.y / d);
            }
            if (t == 0) X[(int64_t)j * ld + j] = make_double2(1.0, 0.0);
        }
        if (t == 0) { beta[j] = bj; tau[j] = tj; }
        __syncthreads();
        if (tj == 0.0) continue;
        const int g = t >> 6;
        for (int cb = j + 1; cb < n; cb += 64) {
            const int c = cb + (t & 63);
            double2 w = make_double2(0.0, 0.0);
            if (c < n) {
                for (int i = j + g; i < rows; i += QR_G) {
                    const double2 v = X[(int64_t)i * ld + j];
                    const double2 x = X[(int64_t)i * ld + c];
                    const double2 p = cmulc(v, x);
                    w.x += p.x; w.y += p.y;
                }
            }
            wpart[g * 64 + (t & 63)] = w;
            __syncthreads();
            if (c < n) {
                double2 ws = make_double2(0.0, 0.0);
#pragma unroll
                for (int q = 0; q < QR_G; ++q) { ws.x += wpart[q * 64 + (t & 63)].x; ws.y += wpart[q * 64 + (t & 63)].y; }
                ws.x *= tj; ws.y *= tj;
                for (int i = j + g; i < rows; i += QR_G) {
                    const double2 v = X[(int64_t)i * ld + j];
                    const double2 p = cmul(v, ws);
                    double2 &x = X[(int64_t)i * ld + c];
                    x.x -= p.x; x.y -= p.y;
                }
            }
            __syncthreads();
        }
    }
}

// Y <- H_0 ... H_{k-1} Y for Y (rows x nq, leading dim ldy); reflectors in V
// (rows x k part of a rows x ldv array), tau[k].
__device__ void hh_apply(double2 *Y, int rows, int nq, int ldy, const double2 *V, int ldv, int k,
                         const double *tau, double2 *wpart) {
    const int t = threadIdx.x;
    const int g = t >> 6;
    for (int j = k - 1; j >= 0; --j) {
        const double tj = tau[j];
        if (tj == 0.0) continue;
        for (int cb = 0; cb < nq; cb += 64) {
            const int c = cb + (t & 63);
            double2 w = make_double2(0.0, 0.0);
            if (c < nq) {
                for (int i = j + g; i < rows; i += QR_G) {
                    const double2 v = V[(int64_t)i * ldv + j];
                    const double2 y = Y[(int64_t)i * ldy + c];
                    const double2 p = cmulc(v, y);
                    w.x += p.x; w.y += p.y;
                }
            }
            wpart[g * 64 + (t & 63)] = w;
            __syncthreads();
            if (c < nq) {
                double2 ws = make_double2(0.0, 0.0);
#pragma unroll
                for (int q = 0; q < QR_G; ++q) { ws.x += wpart[q * 64 + (t & 63)].x; ws.y += wpart[q * 64 + (t & 63)].y; }
                ws.x *= tj; ws.y *= tj;
                for (int i = j + g; i < rows; i += QR_G) {
                    const double2 v = V[(int64_t)i * ldv + j];
                    const double2 p = cmul(v, ws);
                    double2 &y = Y[(int64_t)i * ldy + c];
                    y.x -= p.x; y.y -= p.y;
                }
            }
            __syncthreads();
        }
    }
}

struct LeafArgs {
    MatDesc in;              // level input (row i, col j), rows x n
    int rows, n, nb, top;
    char *ws; int64_t ws_bs;  // workspace base and per-batch stride (bytes)
    size_t v_off, t_off, b_off, rs_off;
    MatOut R; int want_r;    // top only: k x n
};

__global__ void __launch_bounds__(QR_NT) k_qr_leaf(LeafArgs a) {
    extern __shared__ double2 lds[];
    __shared__ double red[QR_NT / 64];
    __shared__ double2 wpart[QR_NT];
    __shared__ double2 sbeta[128];  // k <= 90 whenever one block holds the matrix
    __shared__ double stau[128];
    const int blk = blockIdx.x;
    const int bt = blockIdx.y;
    const int r0 = (int)(((int64_t)blk * a.rows) / a.nb);
    const int r1 = (int)(((int64_t)(blk + 1) * a.rows) / a.nb);
    const int len = r1 - r0;
    const int n = a.n;
    double2 *X = lds;
    char *wb = a.ws + (int64_t)bt * a.ws_bs;
    const char *inb = reinterpret_cast<const char *>(a.in.p) + (int64_t)bt * a.in.bs * a.in.esz;
    for (int e = threadIdx.x; e < len * n; e += QR_NT) {
        const int i = e / n, j = e % n;
        X[e] = ld_c(inb, a.in.esz, (int64_t)(r0 + i) * a.in.rs + (int64_t)j * a.in.cs, a.in.conj);
    }
    __syncthreads();
    hh_factor(X, len, n, n, sbeta, stau, red, wpart);
    __syncthreads();
    const int k = len < n ? len : n;
    double2 *Vb = reinterpret_cast<double2 *>(wb + a.v_off) + (int64_t)r0 * n;
    for (int e = threadIdx.x; e < len * n; e += QR_NT) Vb[e] = X[e];
    double *tb = reinterpret_cast<double *>(wb + a.t_off) + (int64_t)blk * n;
    double2 *bb = reinterpret_cast<double2 *>(wb + a.b_off) + (int64_t)blk * n;
    for (int j = threadIdx.x; j < n; j += QR_NT) {
        tb[j] = j < k ? stau[j] : 0.0;
        bb[j] = j < k ? sbeta[j] : make_double2(0.0, 0.0);
    }
    if (!a.top) {
        double2 *Rb = reinterpret_cast<double2 *>(wb + a.rs_off) + (int64_t)blk * n * n;
        for (int e = threadIdx.x; e < n * n; e += QR_NT) {
            const int i = e / n, j = e % n;
            double2 v = make_double2(0.0, 0.0);
            if (i < k) {
                if (j == i) v = sbeta[i];
                else if (j > i) v = X[i * n + j];
            }
            Rb[e] = v;
        }
    } else if (a.want_r) {
        char *rb = reinterpret_cast<char *>(a.R.p) + (int64_t)bt * a.R.bs * a.R.esz;
        for (int e = threadIdx.x; e < k * n; e += QR_NT) {
            const int i = e / n, j = e % n;
            double2 v = make_double2(0.0, 0.0);
            if (j == i) v = sbeta[i];
            else if (j > i) v = X[i * n + j];
            st_c(rb, a.R.esz, (int64_t)i * a.R.rs + (int64_t)j * a.R.cs, v, a.R.conj);
        }
    }
}

struct FormArgs {
    int rows, n, nb, k, top, level0;
    char *ws; int64_t ws_bs;
    size_t v_off, t_off, x_off, q_off;  // x_off: parent Q ((nb n) x k), q_off: this level's Q
    MatOut out;                          // level 0 destination
};

__global__ void __launch_bounds__(QR_NT) k_qr_form(FormArgs a) {
    extern __shared__ double2 lds[];
    __shared__ double2 wpart[QR_NT];
    const int blk = blockIdx.x;
    const int bt = blockIdx.y;
    const int r0 = (int)(((int64_t)blk * a.rows) / a.nb);
    const int r1 = (int)(((int64_t)(blk + 1) * a.rows) / a.nb);
    const int len = r1 - r0;
    const int n = a.n, k = a.k;
    const int kb = len < n ? len : n;
    char *wb = a.ws + (int64_t)bt * a.ws_bs;
    double2 *Y = lds;  // len x k
    const double2 *X = a.top ? nullptr : reinterpret_cast<const double2 *>(wb + a.x_off);
    for (int e = threadIdx.x; e < len * k; e += QR_NT) {
        const int i = e / k, c = e % k;
        double2 v = make_double2(0.0, 0.0);
        if (i < kb) {
            if (a.top) v = make_double2(i == c ? 1.0 : 0.0, 0.0);
            else v = X[((int64_t)blk * n + i) * k + c];
        }
        Y[e] = v;
    }
    __syncthreads();
    const double2 *Vb = reinterpret_cast<const double2 *>(wb + a.v_off) + (int64_t)r0 * n;
    const double *tb = reinterpret_cast<const double *>(wb + a.t_off) + (int64_t)blk * n;
    hh_apply(Y, len, k, k, Vb, n, kb, tb, wpart);
    if (a.level0) {
        char *ob = reinterpret_cast<char *>(a.out.p) + (int64_t)bt * a.out.bs * a.out.esz;
        for (int e = threadIdx.x; e < len * k; e += QR_NT) {
            const int i = e / k, c = e % k;
            st_c(ob, a.out.esz, (int64_t)(r0 + i) * a.out.rs + (int64_t)c * a.out.cs, Y[e], a.out.conj);
        }
    } else {
        double2 *qb = reinterpret_cast<double2 *>(wb + a.q_off) + (int64_t)r0 * k;
        for (int e = threadIdx.x; e < len * k; e += QR_NT) qb[e] = Y[e];
    }
}

// Fallback: one workgroup per matrix, matrix in global workspace.
struct GlobalQrArgs {
    MatDesc in; int m, n;
    char *ws; int64_t ws_bs;
    size_t w_off, y_off, t_off, b_off;
    MatOut Q; MatOut R; int want_r;
    int batch;
    const int *only_if;  // optional [batch]: factor only the items whose flag has bit 4 set
};

// One workgroup per matrix; the workgroups loop over the batch (workspace slot
// = blockIdx.x), skipping the items not flagged in only_if when it is given.
__global__ void __launch_bounds__(QR_NT) k_qr_global(GlobalQrArgs a) {
    __shared__ double red[QR_NT / 64];
    __shared__ double2 wpart[QR_NT];
    const int m = a.m, n = a.n, k = m < n ? m : n;
    char *wb = a.ws + (int64_t)blockIdx.x * a.ws_bs;
    double2 *X = reinterpret_cast<double2 *>(wb + a.w_off);
    double2 *Y = reinterpret_cast<double2 *>(wb + a.y_off);
    double *tau = reinterpret_cast<double *>(wb + a.t_off);
    double2 *beta = reinterpret_cast<double2 *>(wb + a.b_off);
    for (int bt = blockIdx.x; bt < a.batch; bt += gridDim.x) {
        if (a.only_if && !(a.only_if[bt] & 4)) continue;  // uniform over the block
        const char *inb = reinterpret_cast<const char *>(a.in.p) + (int64_t)bt * a.in.bs * a.in.esz;
        __syncthreads();  // the previous item's last reads of the workspace
        for (int64_t e = threadIdx.x; e < (int64_t)m * n; e += QR_NT) {
            const int i = (int)(e / n), j = (int)(e % n);
            X[e] = ld_c(inb, a.in.esz, (int64_t)i * a.in.rs + (int64_t)j * a.in.cs, a.in.conj);
        }
        __syncthreads();
        hh_factor(X, m, n, n, beta, tau, red, wpart);
        __syncthreads();
        for (int64_t e = threadIdx.x; e < (int64_t)m * k; e += QR_NT) {
            const int i = (int)(e / k), c = (int)(e % k);
            Y[e] = make_double2(i == c ? 1.0 : 0.0, 0.0);
        }
        __syncthreads();
        hh_apply(Y, m, k, k, X, n, k, tau, wpart);
        char *qb = reinterpret_cast<char *>(a.Q.p) + (int64_t)bt * a.Q.bs * a.Q.esz;
        for (int64_t e = threadIdx.x; e < (int64_t)m * k; e += QR_NT) {
            const int i = (int)(e / k), c = (int)(e % k);
            st_c(qb, a.Q.esz, (int64_t)i * a.Q.rs + (int64_t)c * a.Q.cs, Y[e], a.Q.conj);
        }
        if (a.want_r) {
            char *rb = reinterpret_cast<char *>(a.R.p) + (int64_t)bt * a.R.bs * a.R.esz;
            for (int64_t e = threadIdx.x; e < (int64_t)k * n; e += QR_NT) {
                const int i = (int)(e / n), j = (int)(e % n);
                double2 v = make_double2(0.0, 0.0);
                if (j == i) v = beta[i];
                else if (j > i) v = X[(int64_t)i * n + j];
                st_c(rb, a.R.esz, (int64_t)i * a.R.rs + (int64_t)j * a.R.cs, v, a.R.conj);
            }
        }
    }
}

struct TsqrLevel {
    int rows, nb;
    size_t v_off, t_off, b_off, rs_off, q_off;  // byte offsets inside one batch item's workspace
};

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// Plans the TSQR tree; returns per-batch workspace bytes.
size_t plan_tsqr(int m, int n, std::vector<TsqrLevel> &lv) {
    lv.clear();
    const int rb = QR_LDS / n;
    int rows = m;
    size_t off = 0;
    auto take = [&](size_t bytes) { size_t o = off; off += align256(bytes); return o; };
    while (true) {
        TsqrLevel L;
        L.rows = rows;
        L.nb = (rows + rb - 1) / rb;
        if (L.nb < 1) L.nb = 1;
        L.v_off = take((size_t)rows * n * 16);
        L.t_off = take((size_t)L.nb * n * 8);
        L.b_off = take((size_t)L.nb * n * 16);
        L.rs_off = (L.nb > 1) ? take((size_t)L.nb * n * n * 16) : 0;
        L.q_off = lv.empty() ? 0 : take((size_t)rows * n * 16);
        lv.push_back(L);
        if (L.nb == 1) break;
        rows = L.nb * n;
    }
    return off;
}

bool use_tsqr(int m, int n) { return n <= 64 || (int64_t)m * n <= QR_LDS; }

size_t global_qr_bytes(int m, int n, size_t *w, size_t *y, size_t *t, size_t *b) {
    const int k = m < n ? m : n;
    size_t off = 0;
    *w = off; off += align256((size_t)m * n * 16);
    *y = off; off += align256((size_t)m * k * 16);
    *t = off; off += align256((size_t)k * 8);
    *b = off; off += align256((size_t)k * 16);
    return off;
}

// ---------------------------------------------------------------- Cholesky + inverse
// One workgroup of 1024 threads per matrix, n <= 64.  Right-looking elimination on
// the augmented pair [W | E] = [G + sI | I]: at pivot k every lower row i takes
//   row_i -= conj(W[k][i]) / W[k][k] * row_k
// on both halves, and row k is scaled by 1 / sqrt(W[k][k]).  With G + sI =
// L D L^H this leaves W = D^{1/2} L^H = R (upper) and E = D^{-1/2} L^{-1} =
// R^{-H} (lower), so R^{-1} = E^H comes out of the same sweep, with no
// back substitution.  Thread (row i, lane q of CL per row) keeps its part of the
// row in registers: W[i][j] for j = i + q + CL m >= i and E[i][j] for
// j = q + CL m <= i (m < NMAX / CL); the owners of row k + 1 publish it to LDS
// (two buffers) for the next pivot: one barrier per pivot.  Sixteen lanes per
// row (1024 threads, four waves per SIMD) hide the latency of the short
// dependent chains.  Rf (optional) receives R.
__device__ inline void csub_conj_mul(double2 &w, double ax, double ay, double2 c) {
    // w -= (ax - i ay) * c, i.e. w -= conj(a) c / d with (ax, ay) = a / d
    w.x = fma(-ax, c.x, w.x);
    w.x = fma(-ay, c.y, w.x);
    w.y = fma(-ax, c.y, w.y);
    w.y = fma(ay, c.x, w.y);
}

// NMAX rows of CL lanes each (64 x 16 = 1024 threads).  G holds nparts
// matrices per batch item ([batch][nparts][n][n]) whose sum is factored.
template <int NMAX, int CL>
__global__ void __launch_bounds__(NMAX * CL) k_chol_inv(const double2 *G, int nparts, int n, double shift,
                                                       double clamp, double2 *Rinv, double2 *Rf, int *flags) {
    constexpr int CT = NMAX * CL;   // threads per matrix
    constexpr int CM = NMAX / CL;   // row elements per lane
    __shared__ double2 PW[2][NMAX];
    __shared__ double2 PE[2][NMAX];
    __shared__ double PD[2][2];  // pivot (raised to the clamp if below it) and its reciprocal
    __shared__ double red[CT / 64];
    const int b = blockIdx.x, t = threadIdx.x;
    const double2 *Gb = G + (int64_t)b * nparts * n * n;
    const int ti = t / CL, tq = t % CL;
    const bool row = ti < n;
    double2 w[CM], e[CM];
#pragma unroll
    for (int m = 0; m < CM; ++m) {
        const int j = ti + tq + CL * m;
        w[m] = make_double2(0.0, 0.0);
        if (row && j < n)
            for (int q = 0; q < nparts; ++q) {  // fixed order: the sum is reproducible
                const double2 g = Gb[((int64_t)q * n + ti) * n + j];
                w[m].x += g.x;
                w[m].y += g.y;
            }
        const int je = tq + CL * m;
        e[m] = make_double2(row && je == ti ? 1.0 : 0.0, 0.0);
    }
    // tr(G) / n
    {
        double v = (row && tq == 0) ? w[0].x : 0.0;
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if ((t & 63) == 0) red[t >> 6] = v;
    }
    __syncthreads();
    double tr = 0.0;
#pragma unroll
    for (int i = 0; i < CT / 64; ++i) tr += red[i];
    const double scale = tr / n;
    const double sh = shift * scale, cl = clamp * scale;
    if (row && tq == 0) w[0].x += sh;
    // the owner of a pivot row publishes the row, the pivot and its reciprocal
    auto publish_pivot = [&](int slot) {
        double d = w[0].x;
        if (!(d >= cl)) {
            if (flags) flags[b] |= 4;
            d = cl > 0.0 ? cl : 1e-300;
        }
        PD[slot][0] = d;
        PD[slot][1] = 1.0 / d;
    };
    if (ti == 0) {
#pragma unroll
        for (int m = 0; m < CM; ++m) {
            const int j = tq + CL * m;
            if (j < n) { PW[0][j] = w[m]; PE[0][j] = e[m]; }
        }
        if (tq == 0) publish_pivot(0);
    }
    __syncthreads();
    double myrk = 1.0;  // 1 / sqrt of this row's pivot
    for (int k = 0; k < n; ++k) {
        const int pb = k & 1;
        const double d = PD[pb][0];
        if (ti == k) {
            myrk = 1.0 / sqrt(d);
            if (tq == 0) w[0] = make_double2(d, 0.0);  // a raised pivot stays consistent
        } else if (row && ti > k) {
            const double inv = PD[pb][1];
            const double2 a = PW[pb][ti];
            const double ax = a.x * inv, ay = a.y * inv;
            double2 cw[CM], ce[CM];
#pragma unroll
            for (int m = 0; m < CM; ++m) {
                const int j = ti + tq + CL * m;
                cw[m] = PW[pb][j < NMAX ? j : NMAX - 1];  // unconditional loads, then select
                ce[m] = PE[pb][tq + CL * m];
            }
#pragma unroll
            for (int m = 0; m < CM; ++m) {
                if (ti + tq + CL * m < n) csub_conj_mul(w[m], ax, ay, cw[m]);
                if (tq + CL * m <= k) csub_conj_mul(e[m], ax, ay, ce[m]);
            }
            if (ti == k + 1) {
#pragma unroll
                for (int m = 0; m < CM; ++m) {
                    const int j = tq + CL * m;
                    if (ti + j < n) PW[pb ^ 1][ti + j] = w[m];  // column ti + tq + CL m
                    if (j < n) PE[pb ^ 1][j] = e[m];
                }
                if (tq == 0) publish_pivot(pb ^ 1);  // w[0]: the diagonal, final after pivot k
            }
        }
        __syncthreads();
    }
    if (!row) return;
    // R[i][j] = W[i][j] / sqrt(d_i) (j >= i), R^{-1}[j][i] = conj(E[i][j]) / sqrt(d_i) (j <= i)
    double2 *Ob = Rinv + (int64_t)b * n * n;
#pragma unroll
    for (int m = 0; m < CM; ++m) {
        const int j = tq + CL * m;
        if (j < n) Ob[j * n + ti] = j <= ti ? make_double2(e[m].x * myrk, -e[m].y * myrk) : make_double2(0.0, 0.0);
    }
    if (Rf) {
        double2 *Fb = Rf + (int64_t)b * n * n;
#pragma unroll
        for (int m = 0; m < CM; ++m) {
            const int j = ti + tq + CL * m;
            if (j < n) Fb[ti * n + j] = j == ti ? make_double2(w[m].x * myrk, 0.0)
                                                : make_double2(w[m].x * myrk, w[m].y * myrk);
            const int jl = tq + CL * m;
            if (jl < ti) Fb[ti * n + jl] = make_double2(0.0, 0.0);
        }
    }
}

// One pass of CholeskyQR over a block of p.rb rows of a (batch x m x n,
// n <= 64) complex matrix, 256 threads, CQR_ROWS rows staged in LDS at a time:
// the rows are read through p.src's strides (complex64 or complex128,
// conjugated if asked), multiplied by the inverse factor p.Ri of the previous
// pass when given (Y = X Ri, Ri upper triangular), written to the contiguous
// complex128 rows p.X and/or through p.dst's strides, and their Gram matrix
// Y^H Y (upper triangle) is written to p.part[b][block] when p.part is given.
// Each thread of the Gram owns a 4 x 4 block of it; each thread of the product
// owns one row and 8 columns of Y.
__global__ void __launch_bounds__(256) k_cqr_rows(CqrPass p) {
    __shared__ double2 sRi[64][CQR_LD];
    __shared__ double2 sA[CQR_ROWS][CQR_LD];
    __shared__ double2 sY[CQR_ROWS][CQR_LD];
    const int t = threadIdx.x, b = blockIdx.y, n = p.n;
    const int r_beg = blockIdx.x * p.rb, r_end = min(p.m, r_beg + p.rb);
    const bool apply = p.Ri != nullptr;
    if (apply) {  // all loads issued before the LDS stores (n * n <= 16 * 256)
        const double2 *Rb = reinterpret_cast<const double2 *>(p.Ri) + (int64_t)b * n * n;
        double2 rv[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = t + 256 * i;
            rv[i] = e < n * n ? Rb[e] : make_double2(0.0, 0.0);
        }
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const int e = t + 256 * i;
            if (e < n * n) sRi[e / n][e % n] = rv[i];
        }
    }
    const int gi = (t >> 4) * 4, gj = (t & 15) * 4;        // Gram block
    const bool gown = p.part && gi < n && gj < n && gi <= gj + 3;
    double2 g[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) g[i][j] = make_double2(0.0, 0.0);
    const int yr = t >> 3, yc = t & 7;                      // product: row yr, columns yc + 8 q
    const bool by_col = p.s_cs != 1;                        // source contiguous along rows
    for (int r0 = r_beg; r0 < r_end; r0 += CQR_ROWS) {
        const int nr = min(CQR_ROWS, r_end - r0);
        {   // CQR_ROWS * n <= 8 * 256 elements: all loads issued before the LDS stores
            double2 av[8];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = t + 256 * i;
                const int r = by_col ? e % CQR_ROWS : e / n, c = by_col ? e / CQR_ROWS : e % n;
                av[i] = (e < CQR_ROWS * n && r < nr)
                            ? ld_c(p.src, p.s_esz, (int64_t)b * p.s_bs + (int64_t)(r0 + r) * p.s_rs +
                                                       (int64_t)c * p.s_cs, p.s_conj)
                            : make_double2(0.0, 0.0);
            }
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const int e = t + 256 * i;
                const int r = by_col ? e % CQR_ROWS : e / n, c = by_col ? e / CQR_ROWS : e % n;
                if (e < CQR_ROWS * n) sA[r][c] = av[i];
            }
        }
        __syncthreads();
        double2 (*Y)[CQR_LD] = sA;
        if (apply) {
            double2 y[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) y[q] = make_double2(0.0, 0.0);
#pragma unroll 8
            for (int k = 0; k < n; ++k) {
                const double2 a = sA[yr][k];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    const int j = yc + 8 * q;
                    if (j < n && k <= j) {
                        const double2 r = sRi[k][j];
                        y[q].x = fma(a.x, r.x, fma(-a.y, r.y, y[q].x));
                        y[q].y = fma(a.x, r.y, fma(a.y, r.x, y[q].y));
                    }
                }
            }
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int j = yc + 8 * q;
                if (j < n) sY[yr][j] = y[q];
            }
            __syncthreads();
            Y = sY;
        }
        if (p.X)
            for (int e = t; e < nr * n; e += 256) {
                const int r = e / n, c = e % n;
                reinterpret_cast<double2 *>(p.X)[((int64_t)b * p.m + r0 + r) * n + c] = Y[r][c];
            }
        if (p.dst)
            for (int e = t; e < nr * n; e += 256) {
                int r, c;
                if (p.d_cs != 1) { c = e / nr; r = e % nr; }
                else { r = e / n; c = e % n; }
                st_c(p.dst, p.d_esz, (int64_t)b * p.d_bs + (int64_t)(r0 + r) * p.d_rs + (int64_t)c * p.d_cs, Y[r][c],
                     p.d_conj);
            }
        if (gown)
            for (int r = 0; r < nr; ++r) {
                double2 xi[4], xj[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    xi[i] = Y[r][gi + i < n ? gi + i : 0];
                    xj[i] = Y[r][gj + i < n ? gj + i : 0];
                }
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < 4; ++j) {  // conj(x_i) x_j
                        g[i][j].x = fma(xi[i].x, xj[j].x, fma(xi[i].y, xj[j].y, g[i][j].x));
                        g[i][j].y = fma(xi[i].x, xj[j].y, fma(-xi[i].y, xj[j].x, g[i][j].y));
                    }
            }
        __syncthreads();
    }
    if (gown) {
        double2 *P = reinterpret_cast<double2 *>(p.part) + ((int64_t)b * gridDim.x + blockIdx.x) * n * n;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int j = 0; j < 4; ++j)
                if (gi + i < n && gj + j < n) P[(gi + i) * n + gj + j] = g[i][j];
    }
}

// G[b][e] = sum over p of parts[b][p][e] (e < nn), in a fixed order: 256
// threads per SUM_E entries, each of the 256 / SUM_E slices sums the parts
// p = slice, slice + slices, ... in order, then the slices are added in order.
__global__ void __launch_bounds__(256) k_sum_parts(const double2 *parts, int nparts, int nn, double2 *G) {
    constexpr int SL = 256 / SUM_E;
    __shared__ double2 red[SL][SUM_E];
    const int t = threadIdx.x, b = blockIdx.y;
    const int el = t % SUM_E, sl = t / SUM_E;
    const int e = blockIdx.x * SUM_E + el;
    double2 acc = make_double2(0.0, 0.0);
    if (e < nn) {
        const double2 *P = parts + (int64_t)b * nparts * nn + e;
        for (int q = sl; q < nparts; q += SL) {
            const double2 v = P[(int64_t)q * nn];
            acc.x += v.x;
            acc.y += v.y;
        }
    }
    red[sl][el] = acc;
    __syncthreads();
    if (sl == 0 && e < nn) {
        double2 r = red[0][el];
        for (int q = 1; q < SL; ++q) {
            r.x += red[q][el].x;
            r.y += red[q][el].y;
        }
        G[(int64_t)b * nn + e] = r;
    }
}

// x[i] *= (re + i im), complex128.
__global__ void __launch_bounds__(256) k_scale(double2 *x, int64_t n, double re, double im) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double2 v = x[i];
        x[i] = make_double2(v.x * re - v.y * im, v.x * im + v.y * re);
    }
}

__global__ void __launch_bounds__(256) k_strided_copy(const char *in, int ie, int64_t ibs, int64_t irs, int64_t ics,
                                                     char *out, int oe, int64_t obs, int64_t ors, int64_t ocs, int m,
                                                     int n, int batch, int conj) {
    const int64_t per = (int64_t)m * n, total = per * batch;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int b = (int)(e / per);
        const int64_t r = e - (int64_t)b * per;
        const int i = (int)(r / n), j = (int)(r - (int64_t)i * n);
        double2 v = ld_c(in, ie, (int64_t)b * ibs + (int64_t)i * irs + (int64_t)j * ics, conj);
        st_c(out, oe, (int64_t)b * obs + (int64_t)i * ors + (int64_t)j * ocs, v, 0);
    }
}

}  // namespace

hipError_t launch_chol_inv(const double *G, int n, int batch, double shift, double clamp, double *Rinv, double *Rf,
                           int *flags, hipStream_t s) {
    if (n > 64 || n < 1) return hipErrorInvalidValue;
    const double2 *g = reinterpret_cast<const double2 *>(G);
    double2 *ri = reinterpret_cast<double2 *>(Rinv), *rf = reinterpret_cast<double2 *>(Rf);
    hipLaunchKernelGGL((k_chol_inv<64, 16>), dim3(batch), dim3(1024), 0, s, g, 1, n, shift, clamp, ri, rf, flags);
    return hipGetLastError();
}

int cqr_rows_per_block(int m) {
    // one staged chunk per workgroup (the passes are latency-bound: more
    // workgroups, each with a short chain), at most 1024 blocks per matrix
    const int per = (m + 1023) / 1024;
    return std::max(CQR_ROWS, (per + CQR_ROWS - 1) / CQR_ROWS * CQR_ROWS);
}

hipError_t launch_sum_parts(const double *parts, int nparts, int n, int batch, double *G, hipStream_t s) {
    if (n < 1 || nparts < 1 || batch < 1) return hipSuccess;
    if (batch > 65535) return hipErrorInvalidValue;
    const int nn = n * n;
    hipLaunchKernelGGL(k_sum_parts, dim3((nn + SUM_E - 1) / SUM_E, batch), dim3(256), 0, s,
                       reinterpret_cast<const double2 *>(parts), nparts, nn, reinterpret_cast<double2 *>(G));
    return hipGetLastError();
}

hipError_t launch_cqr_pass(const CqrPass &p, hipStream_t s) {
    if (p.m <= 0 || p.batch <= 0) return hipSuccess;
    if (p.n < 1 || p.n > 64 || p.rb < CQR_ROWS || p.rb % CQR_ROWS) return hipErrorInvalidValue;
    if (p.batch > 65535) return hipErrorInvalidValue;
    const int nblk = (p.m + p.rb - 1) / p.rb;
    hipLaunchKernelGGL(k_cqr_rows, dim3(nblk, p.batch), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_scale(void *x, int64_t n, double re, double im, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_scale, dim3((unsigned)g), dim3(256), 0, s, reinterpret_cast<double2 *>(x), n, re, im);
    return hipGetLastError();
}

hipError_t launch_strided_copy(const void *in, int ie, int64_t ibs, int64_t irs, int64_t ics, void *out, int oe,
                               int64_t obs, int64_t ors, int64_t ocs, int m, int n, int batch, int conj,
                               hipStream_t s) {
    const int64_t total = (int64_t)m * n * batch;
    if (total <= 0) return hipSuccess;
    int64_t g = (total + 255) / 256;
    if (g > 4096) g = 4096;
    hipLaunchKernelGGL(k_strided_copy, dim3((unsigned)g), dim3(256), 0, s, reinterpret_cast<const char *>(in), ie, ibs,
                       irs, ics, reinterpret_cast<char *>(out), oe, obs, ors, ocs, m, n, batch, conj);
    return hipGetLastError();
}

// workgroups (and workspace slots) of the fallback: at most 512, and at most
// 16 MiB of workspace (at least one slot)
static int qr_fallback_slots(int m, int n, int batch) {
    size_t w, y, t, b;
    const size_t per = global_qr_bytes(m, n, &w, &y, &t, &b);
    const size_t cap = (size_t)16 << 20;
    const int by_cap = (int)std::max<size_t>(1, cap / std::max<size_t>(per, 1));
    return std::max(1, std::min(std::min(batch, 512), by_cap));
}

size_t qr_fallback_workspace_bytes(int m, int n, int batch) {
    if (m <= 0 || n <= 0 || batch <= 0) return 0;
    size_t w, y, t, b;
    return global_qr_bytes(m, n, &w, &y, &t, &b) * (size_t)qr_fallback_slots(m, n, batch);
}

hipError_t launch_qr_fallback(const QrArgs &q, const int *flags, void *workspace, hipStream_t s) {
    const int m = q.m, n = q.n;
    if (m <= 0 || n <= 0 || q.batch <= 0) return hipSuccess;
    if (!flags || !workspace) return hipErrorInvalidValue;
    GlobalQrArgs g;
    const size_t per = global_qr_bytes(m, n, &g.w_off, &g.y_off, &g.t_off, &g.b_off);
    g.in = MatDesc{q.A, q.a_esz, q.a_bs, q.a_rs, q.a_cs, q.a_conj};
    g.m = m; g.n = n; g.ws = reinterpret_cast<char *>(workspace); g.ws_bs = (int64_t)per;
    g.Q = MatOut{q.Q, q.q_esz, q.q_bs, q.q_rs, q.q_cs, q.q_conj};
    g.R = MatOut{q.R, q.r_esz, q.r_bs, q.r_rs, q.r_cs, q.r_conj};
    g.want_r = q.R != nullptr;
    g.batch = q.batch;
    g.only_if = flags;
    hipLaunchKernelGGL(k_qr_global, dim3(qr_fallback_slots(m, n, q.batch)), dim3(QR_NT), 0, s, g);
    return hipGetLastError();
}

size_t qr_workspace_bytes(int m, int n, int batch) {
    if (m <= 0 || n <= 0) return 0;
    std::vector<TsqrLevel> lv;
    size_t w, y, t, b;
    const size_t per = use_tsqr(m, n) ? plan_tsqr(m, n, lv) : global_qr_bytes(m, n, &w, &y, &t, &b);
    return per * (size_t)batch;
}

hipError_t launch_qr(const QrArgs &q, void *workspace, hipStream_t s) {
    const int m = q.m, n = q.n;
    if (m <= 0 || n <= 0 || q.batch <= 0) return hipSuccess;
    const int k = m < n ? m : n;
    char *ws = reinterpret_cast<char *>(workspace);
    MatDesc in{q.A, q.a_esz, q.a_bs, q.a_rs, q.a_cs, q.a_conj};
    MatOut qo{q.Q, q.q_esz, q.q_bs, q.q_rs, q.q_cs, q.q_conj};
    MatOut ro{q.R, q.r_esz, q.r_bs, q.r_rs, q.r_cs, q.r_conj};
    if (!use_tsqr(m, n)) {
        GlobalQrArgs g;
        const size_t per = global_qr_bytes(m, n, &g.w_off, &g.y_off, &g.t_off, &g.b_off);
        g.in = in; g.m = m; g.n = n; g.ws = ws; g.ws_bs = (int64_t)per;
        g.Q = qo; g.R = ro; g.want_r = q.R != nullptr;
        g.batch = q.batch;
        g.only_if = nullptr;
        hipLaunchKernelGGL(k_qr_global, dim3(q.batch), dim3(QR_NT), 0, s, g);
        return hipGetLastError();
    }
    std::vector<TsqrLevel> lv;
    const size_t per = plan_tsqr(m, n, lv);
    const size_t lds_bytes = (size_t)QR_LDS * 16;
    static bool attr_set = false;
    if (!attr_set) {
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_qr_leaf),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        (void)hipFuncSetAttribute(reinterpret_cast<const void *>(k_qr_form),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bytes);
        attr_set = true;
    }
    for (size_t L = 0; L < lv.size(); ++L) {
        LeafArgs a;
        if (L == 0) a.in = in;
        else a.in = MatDesc{ws + lv[L - 1].rs_off, 16, (int64_t)(per / 16), n, 1, 0};
        a.rows = lv[L].rows; a.n = n; a.nb = lv[L].nb; a.top = (L + 1 == lv.size());
        a.ws = ws; a.ws_bs = (int64_t)per;
        a.v_off = lv[L].v_off; a.t_off = lv[L].t_off; a.b_off = lv[L].b_off; a.rs_off = lv[L].rs_off;
        a.R = ro; a.want_r = (q.R != nullptr);
        hipLaunchKernelGGL(k_qr_leaf, dim3(lv[L].nb, q.batch), dim3(QR_NT), lds_bytes, s, a);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    for (int L = (int)lv.size() - 1; L >= 0; --L) {
        FormArgs f;
        f.rows = lv[L].rows; f.n = n; f.nb = lv[L].nb; f.k = k;
        f.top = (L + 1 == (int)lv.size()); f.level0 = (L == 0);
        f.ws = ws; f.ws_bs = (int64_t)per;
        f.v_off = lv[L].v_off; f.t_off = lv[L].t_off;
        f.x_off = f.top ? 0 : lv[L + 1].q_off;
        f.q_off = lv[L].q_off;
        f.out = qo;
        hipLaunchKernelGGL(k_qr_form, dim3(lv[L].nb, q.batch), dim3(QR_NT), lds_bytes, s, f);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace tnk
