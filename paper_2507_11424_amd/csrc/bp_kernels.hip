// Kernels of belief propagation on the norm network and of the loop BP error
// (Methods, BP contraction and Eqs. avBPError / loopBPerror; Appendix, the
// message update rule and "Computing the BP Error").  All arithmetic FP64
// complex (double2).  The contractions of the message updates run on the
// GETT engine; these kernels embed the site tensors in a uniform padded
// layout, normalise and exchange the messages, form the BP free energy, gather
// the loop matrices and find their eigenvalues.
#include <hip/hip_runtime.h>

#include "kernels.hpp"

namespace tnk {
namespace {

constexpr int NT = 256;

__device__ inline double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ inline double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ inline double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ inline double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ inline double2 cconj(double2 a) { return make_double2(a.x, -a.y); }
__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }
__device__ inline double cabsv(double2 a) { return hypot(a.x, a.y); }
__device__ inline double2 cdiv(double2 a, double2 b) {
    const double d = cabs2(b);
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}
__device__ inline double2 csqrt(double2 z) {
    const double r = cabsv(z);
    if (r == 0.0) return make_double2(0.0, 0.0);
    double x = sqrt(0.5 * (r + fabs(z.x)));
    double y = 0.5 * z.y / x;
    if (z.x >= 0.0) return make_double2(x, y);
    if (z.y < 0.0) { x = -x; y = -y; }
    return make_double2(fabs(y), x);  // sqrt for Re z < 0: (|Im|/(2x), sign(Im) x)
}

__device__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ double block_max(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = NT / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

// One message per block b = z * 4 + leg (legs 0..3 = up, left, down, right):
// the message site z sends through `leg`, out[leg][z] (Dm x Dm), becomes its
// Hermitian part divided by its Frobenius norm and is stored as the message
// into the neighbour w = nbr[z][leg] through the opposite leg; dmax[b] is the
// largest element change (0 for legs without a bond).
__global__ void __launch_bounds__(NT) k_bp_update(const double2 *out, double2 *msg, const int *nbr, int N, int Dm,
                                                 double *dmax) {
    __shared__ double red[NT];
    const int b = blockIdx.x;
    const int z = b >> 2, leg = b & 3;
    const int w = nbr[b];
    if (w < 0) {
        if (threadIdx.x == 0) dmax[b] = 0.0;
        return;
    }
    const int n2 = Dm * Dm;
    const double2 *m = out + ((int64_t)leg * N + z) * n2;
    double2 *dst = msg + ((int64_t)w * 4 + ((leg + 2) & 3)) * n2;
    double s = 0.0;
    for (int e = threadIdx.x; e < n2; e += NT) {
        const int i = e / Dm, j = e % Dm;
        const double2 h = cscale(cadd(m[i * Dm + j], cconj(m[j * Dm + i])), 0.5);
        s += cabs2(h);
    }
    s = block_sum(s, red);
    const double inv = s > 0.0 ? 1.0 / sqrt(s) : 0.0;
    double dm = 0.0;
    for (int e = threadIdx.x; e < n2; e += NT) {
        const int i = e / Dm, j = e % Dm;
        const double2 h = cscale(cadd(m[i * Dm + j], cconj(m[j * Dm + i])), 0.5 * inv);
        const double2 o = dst[e];
        dm = fmax(dm, fmax(fabs(h.x - o.x), fabs(h.y - o.y)));
        dst[e] = h;
    }
    dm = block_max(dm, red);
    if (threadIdx.x == 0) dmax[b] = (s > 0.0 && isfinite(s)) ? dm : INFINITY;
}

__global__ void __launch_bounds__(NT) k_max(const double *x, int n, double *out) {
    __shared__ double red[NT];
    double m = 0.0;
    for (int i = threadIdx.x; i < n; i += NT) m = fmax(m, x[i]);
    m = block_max(m, red);
    if (threadIdx.x == 0) *out = m;
}

// Per site z: zv[z] = sum_ij outr[z][i][j] msg[z][right][i][j] (the pair closed
// with all four messages); ze[z][0 / 1] = sum_ij msg[z][right / down] *
// msg[w][left / up] for the bond to the right / below (1 if absent).
__global__ void __launch_bounds__(NT) k_bp_values(const double2 *outr, const double2 *msg, const int *nbr, int N,
                                                 int Dm, double2 *zv, double2 *ze) {
    __shared__ double red[NT];
    const int z = blockIdx.x;
    const int n2 = Dm * Dm;
    const double2 *o = outr + (int64_t)z * n2;
    const double2 *mr = msg + ((int64_t)z * 4 + 3) * n2;
    double2 acc = make_double2(0.0, 0.0);
    for (int e = threadIdx.x; e < n2; e += NT) acc = cadd(acc, cmul(o[e], mr[e]));
    const double vr = block_sum(acc.x, red), vi = block_sum(acc.y, red);
    if (threadIdx.x == 0) zv[z] = make_double2(vr, vi);
    for (int k = 0; k < 2; ++k) {
        const int leg = k == 0 ? 3 : 2;  // right, down
        const int w = nbr[z * 4 + leg];
        double2 a = make_double2(0.0, 0.0);
        if (w >= 0) {
            const double2 *m1 = msg + ((int64_t)z * 4 + leg) * n2;
            const double2 *m2 = msg + ((int64_t)w * 4 + ((leg + 2) & 3)) * n2;
            for (int e = threadIdx.x; e < n2; e += NT) a = cadd(a, cmul(m1[e], m2[e]));
        }
        const double er = block_sum(a.x, red), ei = block_sum(a.y, red);
        if (threadIdx.x == 0) ze[z * 2 + k] = w >= 0 ? make_double2(er, ei) : make_double2(1.0, 0.0);
    }
}

// out[0] = sum log|zv| - sum log|ze|, out[1] = the same sum of phases, in a
// fixed order (one thread).
__global__ void k_bp_logsum(const double2 *zv, const double2 *ze, int N, double *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double lz = 0.0, ph = 0.0;
    for (int z = 0; z < N; ++z) {
        lz += log(cabsv(zv[z]));
        ph += atan2(zv[z].y, zv[z].x);
        for (int k = 0; k < 2; ++k) {
            const double2 e = ze[z * 2 + k];
            lz -= log(cabsv(e));
            ph -= atan2(e.y, e.x);
        }
    }
    out[0] = lz;
    out[1] = remainder(ph, 2.0 * M_PI);
}

// mats[q] (n x n, n = Dm^2) <- the pair tensor tab[q] = (buffer offset, flag):
// flag 0 copies [i][j], flag 1 transposes.
__global__ void __launch_bounds__(NT) k_gather_mats(const double2 *pairs, const int64_t *off, const int *trans,
                                                   int n, double2 *mats) {
    const int q = blockIdx.x;
    const double2 *src = pairs + off[q];
    double2 *dst = mats + (int64_t)q * n * n;
    const int t = trans[q];
    for (int e = threadIdx.x; e < n * n; e += NT) {
        const int i = e / n, j = e % n;
        dst[e] = t ? src[(int64_t)j * n + i] : src[e];
    }
}

// Eigenvalues of one general complex n x n matrix per lane (the matrix is
// overwritten): Householder reduction to upper Hessenberg form, then the
// shifted QR algorithm with Givens rotations on the active window, Wilkinson
// shifts (an exceptional shift every 11th iteration without deflation) and
// deflation when |h[k][k-1]| <= eps (|h[k][k]| + |h[k-1][k-1]|) (Golub and Van
// Loan, Matrix Computations, 7.4-7.5).  eps[q] = 1 - max|lambda| / sum|lambda|;
// info[q] = 0, or 1 if the iteration limit (30 n per eigenvalue) was hit.
__global__ void k_eig(double2 *mats, int n, int batch, double2 *lam, double *eps, int *info) {
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= batch) return;
    double2 *H = mats + (int64_t)q * n * n;
    double2 *L = lam + (int64_t)q * n;
#define AT(i, j) H[(int64_t)(i) * n + (j)]
    // Householder to Hessenberg: zero H[k+2.., k]
    for (int k = 0; k + 2 < n; ++k) {
        double xn2 = 0.0;
        for (int i = k + 1; i < n; ++i) xn2 += cabs2(AT(i, k));
        const double xn = sqrt(xn2);
        const double2 x0 = AT(k + 1, k);
        const double a0 = cabsv(x0);
        if (xn == 0.0 || xn2 - a0 * a0 <= 1e-300) continue;
        const double2 ph = a0 > 0.0 ? cscale(x0, 1.0 / a0) : make_double2(1.0, 0.0);
        // v = x + ph |x| e1, H <- (I - 2 v v^H / v^H v) H (I - ...)
        const double2 v0 = cadd(x0, cscale(ph, xn));
        double vn2 = cabs2(v0);
        for (int i = k + 2; i < n; ++i) vn2 += cabs2(AT(i, k));
        const double beta = 2.0 / vn2;
        auto v = [&](int i) { return i == k + 1 ? v0 : AT(i, k); };
        // left: rows k+1..n-1, columns k+1..n-1 (column k handled below)
        for (int j = k + 1; j < n; ++j) {
            double2 s = make_double2(0.0, 0.0);
            for (int i = k + 1; i < n; ++i) s = cadd(s, cmul(cconj(v(i)), AT(i, j)));
            s = cscale(s, beta);
            for (int i = k + 1; i < n; ++i) AT(i, j) = csub(AT(i, j), cmul(v(i), s));
        }
        // right: all rows, columns k+1..n-1
        for (int i = 0; i < n; ++i) {
            double2 s = make_double2(0.0, 0.0);
            for (int j = k + 1; j < n; ++j) s = cadd(s, cmul(AT(i, j), v(j)));
            s = cscale(s, beta);
            for (int j = k + 1; j < n; ++j) AT(i, j) = csub(AT(i, j), cmul(s, cconj(v(j))));
        }
        // column k: x -> -ph |x| e1 (v's entries are stored there until now)
        AT(k + 1, k) = cscale(ph, -xn);
        for (int i = k + 2; i < n; ++i) AT(i, k) = make_double2(0.0, 0.0);
    }
    int hi = n - 1, iter = 0, bad = 0;
    const double ulp = 2.220446049250313e-16;
    while (hi >= 0) {
        if (hi == 0) {
            L[0] = AT(0, 0);
            break;
        }
        int l = hi;
        while (l > 0) {
            const double s = cabsv(AT(l, l)) + cabsv(AT(l - 1, l - 1));
            if (cabsv(AT(l, l - 1)) <= ulp * (s > 0.0 ? s : 1.0)) {
                AT(l, l - 1) = make_double2(0.0, 0.0);
                break;
            }
            --l;
        }
        if (l == hi) {
            L[hi] = AT(hi, hi);
            --hi;
            iter = 0;
            continue;
        }
        if (++iter > 30 * n) {
            bad = 1;
            for (int i = 0; i <= hi; ++i) L[i] = AT(i, i);
            break;
        }
        // Wilkinson shift: eigenvalue of the trailing 2x2 closer to h[hi][hi]
        double2 mu;
        if (iter % 11 == 0) {
            mu = cadd(AT(hi, hi), make_double2(0.75 * cabsv(AT(hi, hi - 1)), 0.0));
        } else {
            const double2 a = AT(hi - 1, hi - 1), b = AT(hi - 1, hi), c = AT(hi, hi - 1), d = AT(hi, hi);
            const double2 tr2 = cscale(cadd(a, d), 0.5);
            const double2 dd = cscale(csub(a, d), 0.5);
            const double2 disc = csqrt(cadd(cmul(dd, dd), cmul(b, c)));
            const double2 m1 = cadd(tr2, disc), m2 = csub(tr2, disc);
            mu = cabs2(csub(m1, d)) < cabs2(csub(m2, d)) ? m1 : m2;
        }
        // one QR step on the window l..hi: H - mu I = Q R, H <- R Q + mu I, by
        // Givens rotations G_k on rows (k, k+1), applied to columns as they go
        for (int i = l; i <= hi; ++i) AT(i, i) = csub(AT(i, i), mu);
        for (int k = l; k < hi; ++k) {
            const double2 x = AT(k, k), y = AT(k + 1, k);
            const double r = sqrt(cabs2(x) + cabs2(y));
            double c;
            double2 s;
            if (r == 0.0) {
                c = 1.0;
                s = make_double2(0.0, 0.0);
            } else {
                const double ax = cabsv(x);
                if (ax == 0.0) {
                    c = 0.0;
                    s = cdiv(cconj(y), make_double2(cabsv(y), 0.0));  // phase of conj(y)
                } else {
                    c = ax / r;
                    const double2 ph = cscale(x, 1.0 / ax);          // x / |x|
                    s = cscale(cmul(ph, cconj(y)), 1.0 / r);          // (x/|x|) conj(y) / r
                }
            }
            // rows k, k+1 of columns k..hi: [c, s; -conj(s), c]
            for (int j = k; j <= hi; ++j) {
                const double2 hk = AT(k, j), hk1 = AT(k + 1, j);
                AT(k, j) = cadd(cscale(hk, c), cmul(s, hk1));
                AT(k + 1, j) = csub(cscale(hk1, c), cmul(cconj(s), hk));
            }
            // keep the rotation for the right multiplication: store c, s in the
            // now-zero subdiagonal slot (real c) and in the lambda buffer (s)
            AT(k + 1, k) = make_double2(c, 0.0);
            L[k] = s;
        }
        // H <- R G_l^H ... G_{hi-1}^H: columns k, k+1 of rows l..k+1 (R is upper
        // triangular there; row k+2 still holds the stored cosine of G_{k+1})
        for (int k = l; k < hi; ++k) {
            const double c = AT(k + 1, k).x;
            const double2 s = L[k];
            AT(k + 1, k) = make_double2(0.0, 0.0);
            for (int i = l; i <= k + 1; ++i) {
                const double2 hk = AT(i, k), hk1 = AT(i, k + 1);
                AT(i, k) = cadd(cscale(hk, c), cmul(hk1, cconj(s)));
                AT(i, k + 1) = csub(cscale(hk1, c), cmul(hk, s));
            }
        }
        for (int i = l; i <= hi; ++i) AT(i, i) = cadd(AT(i, i), mu);
    }
#undef AT
    double mx = 0.0, sm = 0.0;
    for (int i = 0; i < n; ++i) {
        const double a = cabsv(L[i]);
        mx = fmax(mx, a);
        sm += a;
    }
    eps[q] = sm > 0.0 ? 1.0 - mx / sm : 0.0;
    info[q] = bad;
}

}  // namespace

hipError_t launch_bp_update(const void *out, void *msg, const int *nbr, int N, int Dm, double *dmax, double *delta,
                            hipStream_t s) {
    hipLaunchKernelGGL(k_bp_update, dim3(N * 4), dim3(NT), 0, s, static_cast<const double2 *>(out),
                       static_cast<double2 *>(msg), nbr, N, Dm, dmax);
    hipLaunchKernelGGL(k_max, dim3(1), dim3(NT), 0, s, dmax, N * 4, delta);
    return hipGetLastError();
}

hipError_t launch_bp_free_energy(const void *outr, const void *msg, const int *nbr, int N, int Dm, void *zv,
                                 void *ze, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_bp_values, dim3(N), dim3(NT), 0, s, static_cast<const double2 *>(outr),
                       static_cast<const double2 *>(msg), nbr, N, Dm, static_cast<double2 *>(zv),
                       static_cast<double2 *>(ze));
    hipLaunchKernelGGL(k_bp_logsum, dim3(1), dim3(64), 0, s, static_cast<const double2 *>(zv),
                       static_cast<const double2 *>(ze), N, out);
    return hipGetLastError();
}

hipError_t launch_gather_mats(const void *pairs, const int64_t *off, const int *trans, int count, int n, void *mats,
                              hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather_mats, dim3(count), dim3(NT), 0, s, static_cast<const double2 *>(pairs), off, trans, n,
                       static_cast<double2 *>(mats));
    return hipGetLastError();
}

hipError_t launch_eig(void *mats, int n, int batch, void *lam, double *eps, int *info, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eig, dim3((batch + 63) / 64), dim3(64), 0, s, static_cast<double2 *>(mats), n, batch,
                       static_cast<double2 *>(lam), eps, info);
    return hipGetLastError();
}

}  // namespace tnk
