// Batched FP64 SVD with truncation by discarded weight, for the adaptive bond
// of the sampler's amplitude boundary.
//
// Each n x n complex matrix R (n <= SVD_NMAX) is diagonalised by one-sided
// (Hestenes) Jacobi: column pairs (p, q) are rotated until every pair is
// orthogonal to a relative tolerance, giving R V = W with orthogonal columns,
// sigma_j = ||w_j||, R = U diag(sigma) V^H with u_j = w_j / sigma_j.  One
// workgroup owns one matrix; a round of the round-robin tournament rotates n/2
// disjoint pairs at once, each pair by a group of lanes that reduce its three
// inner products with cross-lane shuffles.  Matrices with n <= 64 live in LDS
// (W and V, 128 KiB), larger ones in a global workspace slice of the block.
//
// Complex rotation of a pair: with alpha = ||w_p||^2, beta = ||w_q||^2,
// gamma = w_p^H w_q = |gamma| e^{i phi}, the column y = w_q e^{-i phi} has a
// real inner product |gamma| with w_p, and the real Jacobi rotation with
// zeta = (beta - alpha) / (2 |gamma|), t = sign(zeta) / (|zeta| + sqrt(1 + zeta^2)),
// c = 1 / sqrt(1 + t^2), s = c t maps (w_p, y) to (c w_p - s y, s w_p + c y),
// which are orthogonal.
#include "kernels.hpp"

#include <cmath>

namespace tnk {
namespace {

constexpr int SVD_NT = 256;       // threads per matrix held in LDS
constexpr int SVD_NT_GLOBAL = 1024;  // threads per matrix held in global memory (more lanes per column pair)
constexpr int SVD_LDS_N = 64;     // largest n kept in LDS
constexpr int SVD_MAX_SWEEPS = 40;
constexpr double SVD_TOL = 1e-15;  // |gamma| <= tol sqrt(alpha beta) counts as orthogonal
constexpr int SVD_GRID = 512;      // blocks (and workspace slices) at most
constexpr double SVD_RANK_RTOL = 1e-12;  // sigma <= rtol sigma_max counts as zero
// Columns with ||w||^2 <= SVD_NEGL ||R||_F^2 take part in no rotation: they lie
// below the rank cut (sigma_max >= ||R||_F / sqrt(n) >= ||R||_F / 16), and rotating such
// residue against the large columns only drives it towards underflow.
constexpr double SVD_NEGL = 1e-28;
static_assert(SVD_NMAX <= SVD_NT && SVD_NMAX <= SVD_NT_GLOBAL, "the rank sort gives one thread per column");

__device__ inline double2 cm(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }

// Sum over the `w` lanes of an aligned lane group (w a power of two <= 64).
__device__ inline double group_sum(double v, int w) {
    for (int o = w >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

struct SvdArgs {
    const double2 *R; int n, batch;
    double cutoff; int chi_min;
    void *U; void *SV; int esz;
    int *kout;
    double2 *ws;
    int chi_max;    // > 0: at most this many values kept
    double *disc;   // optional [batch]: discarded weight sum_{j>=k} sigma_j^2 / sum_j sigma_j^2
};

__device__ inline void store(void *base, int esz, int64_t off, double2 v) {
    if (esz == 16) reinterpret_cast<double2 *>(base)[off] = v;
    else reinterpret_cast<float2 *>(base)[off] = make_float2((float)v.x, (float)v.y);
}

template <bool IN_LDS, int NT>
__global__ void __launch_bounds__(NT) k_svd_trunc(SvdArgs a) {
    extern __shared__ double2 lds[];
    __shared__ double sig[SVD_NMAX];
    __shared__ double wsort[SVD_NMAX];
    __shared__ double ssort[SVD_NMAX];
    __shared__ int rk[SVD_NMAX];
    __shared__ int rotated;
    __shared__ int kkeep;
    __shared__ double fro2p[NT / 64];
    const int n = a.n, tid = threadIdx.x;
    double2 *W, *V;  // column-major: column j at [j * n]
    if constexpr (IN_LDS) {
        W = lds;
        V = lds + n * n;
    } else {
        W = a.ws + (int64_t)blockIdx.x * 2 * n * n;
        V = W + n * n;
    }
    const int N = n + (n & 1);  // tournament players; index n is a bye when n is odd
    const int P = N / 2;
    int tpp = 64;
    while (tpp > 1 && tpp * P > NT) tpp >>= 1;
    const int pair = tid / tpp, lane = tid % tpp;
    const int NG = NT / tpp;  // lane groups

    for (int b = blockIdx.x; b < a.batch; b += gridDim.x) {
        const double2 *Rb = a.R + (int64_t)b * n * n;
        double f2 = 0;
        for (int e = tid; e < n * n; e += NT) {
            const int i = e / n, j = e % n;
            const double2 x = Rb[e];
            f2 += x.x * x.x + x.y * x.y;
            W[j * n + i] = x;
            V[j * n + i] = make_double2(i == j ? 1.0 : 0.0, 0.0);
        }
        f2 = group_sum(f2, 64);
        if ((tid & 63) == 0) fro2p[tid >> 6] = f2;
        __syncthreads();
        double fro2 = 0;
        for (int w = 0; w < NT / 64; ++w) fro2 += fro2p[w];
        const double negl = SVD_NEGL * fro2;
        for (int sweep = 0; sweep < SVD_MAX_SWEEPS; ++sweep) {
            if (tid == 0) rotated = 0;
            __syncthreads();
            for (int r = 0; r + 1 < N; ++r) {
                int p, q;
                if (pair == 0) { p = N - 1; q = r; }
                else { p = (r + pair) % (N - 1); q = (r - pair + N - 1) % (N - 1); }
                const bool live = pair < P && p < n && q < n;
                double al = 0, be = 0, gr = 0, gi = 0;
                if (live) {
                    for (int i = lane; i < n; i += tpp) {
                        const double2 x = W[p * n + i], y = W[q * n + i];
                        al += x.x * x.x + x.y * x.y;
                        be += y.x * y.x + y.y * y.y;
                        gr += x.x * y.x + x.y * y.y;  // conj(x) y
                        gi += x.x * y.y - x.y * y.x;
                    }
                }
                al = group_sum(al, tpp);
                be = group_sum(be, tpp);
                gr = group_sum(gr, tpp);
                gi = group_sum(gi, tpp);
                const double g = hypot(gr, gi);
                if (live && al > negl && be > negl && g > SVD_TOL * sqrt(al) * sqrt(be)) {
                    const double zeta = (be - al) / (2.0 * g);
                    const double t = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
                    const double c = 1.0 / sqrt(1.0 + t * t), s = c * t;
                    const double2 ph = make_double2(gr / g, -gi / g);  // e^{-i phi}
                    for (int i = lane; i < n; i += tpp) {
                        const double2 x = W[p * n + i], y = cm(W[q * n + i], ph);
                        W[p * n + i] = make_double2(c * x.x - s * y.x, c * x.y - s * y.y);
                        W[q * n + i] = make_double2(s * x.x + c * y.x, s * x.y + c * y.y);
                        const double2 vx = V[p * n + i], vy = cm(V[q * n + i], ph);
                        V[p * n + i] = make_double2(c * vx.x - s * vy.x, c * vx.y - s * vy.y);
                        V[q * n + i] = make_double2(s * vx.x + c * vy.x, s * vx.y + c * vy.y);
                    }
                    if (lane == 0) rotated = 1;
                }
                __syncthreads();
            }
            const int any = rotated;
            __syncthreads();
            if (!any) break;
        }
        // singular values, descending ranks (ties by index)
        for (int j = pair; j < n; j += NG) {
            double v = 0;
            for (int i = lane; i < n; i += tpp) {
                const double2 x = W[j * n + i];
                v += x.x * x.x + x.y * x.y;
            }
            v = group_sum(v, tpp);
            if (lane == 0) sig[j] = sqrt(v);
        }
        __syncthreads();
        if (tid < n) {
            const double sj = sig[tid];
            int c = 0;
            for (int i = 0; i < n; ++i) c += (sig[i] > sj || (sig[i] == sj && i < tid)) ? 1 : 0;
            rk[tid] = c;
            ssort[c] = sj;
            wsort[c] = sj * sj;
        }
        __syncthreads();
        if (tid == 0) {
            // keep rule: fewest values whose discarded tail weight is within
            // cutoff * total, at most the numerical rank, at least min(chi_min, rank)
            int k = 0;
            if (n > 0 && ssort[0] > 0.0) {
                int rank = 0;
                double total = 0;
                for (int j = 0; j < n; ++j) {
                    total += wsort[j];
                    if (ssort[j] > SVD_RANK_RTOL * ssort[0]) ++rank;
                }
                k = rank;
                double tail = 0;
                for (int j = rank - 1; j > 0; --j) {
                    if (tail + wsort[j] > a.cutoff * total) break;
                    tail += wsort[j];
                    k = j;
                }
                const int lo = a.chi_min < rank ? a.chi_min : rank;
                if (k < lo) k = lo;
                if (a.chi_max > 0 && k > a.chi_max) k = a.chi_max;
            }
            kkeep = k;
            a.kout[b] = k;
            if (a.disc) {
                double total = 0, tail = 0;
                for (int j = 0; j < n; ++j) {
                    total += wsort[j];
                    if (j >= k) tail += wsort[j];
                }
                a.disc[b] = total > 0.0 ? tail / total : 0.0;
            }
        }
        __syncthreads();
        const int k = kkeep;
        // U[b](i, rk_j) = w_j(i) / sigma_j; SV[b](rk_j, l) = sigma_j conj(v_j(l)); zero past k
        for (int e = tid; e < n * n; e += NT) {
            const int j = e / n, i = e % n;
            const int col = rk[j];
            const double sj = sig[j];
            double2 u = make_double2(0.0, 0.0), sv = make_double2(0.0, 0.0);
            if (col < k) {
                const double2 w = W[j * n + i], v = V[j * n + i];
                u = make_double2(w.x / sj, w.y / sj);
                sv = make_double2(sj * v.x, -sj * v.y);
            }
            store(a.U, a.esz, (int64_t)b * n * n + (int64_t)i * n + col, u);
            store(a.SV, a.esz, (int64_t)b * n * n + (int64_t)col * n + i, sv);
        }
        __syncthreads();
    }
}

}  // namespace

size_t svd_trunc_workspace_bytes(int n, int batch) {
    if (n <= SVD_LDS_N || batch <= 0) return 0;
    const int grid = batch < SVD_GRID ? batch : SVD_GRID;
    return (size_t)grid * 2 * n * n * sizeof(double2);
}

hipError_t launch_svd_trunc(const double *R, int n, int batch, double cutoff, int chi_min, void *U, void *SV, int esz,
                            int *kout, void *workspace, hipStream_t s, int chi_max, double *disc) {
    if (batch <= 0) return hipSuccess;
    if (n < 1 || n > SVD_NMAX || (esz != 8 && esz != 16)) return hipErrorInvalidValue;
    SvdArgs a;
    a.R = reinterpret_cast<const double2 *>(R);
    a.n = n; a.batch = batch; a.cutoff = cutoff; a.chi_min = chi_min;
    a.U = U; a.SV = SV; a.esz = esz; a.kout = kout;
    a.ws = reinterpret_cast<double2 *>(workspace);
    a.chi_max = chi_max;
    a.disc = disc;
    const int grid = batch < SVD_GRID ? batch : SVD_GRID;
    if (n <= SVD_LDS_N) {
        static bool attr = false;
        const size_t lds = (size_t)2 * SVD_LDS_N * SVD_LDS_N * sizeof(double2);
        if (!attr) {
            const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_svd_trunc<true, SVD_NT>),
                                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            if (e != hipSuccess) return e;
            attr = true;
        }
        hipLaunchKernelGGL((k_svd_trunc<true, SVD_NT>), dim3(grid), dim3(SVD_NT), (size_t)2 * n * n * sizeof(double2), s,
                           a);
    } else {
        if (!workspace) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_svd_trunc<false, SVD_NT_GLOBAL>), dim3(grid), dim3(SVD_NT_GLOBAL), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace tnk
