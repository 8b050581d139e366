// Small kernels around the contraction engine: FP64 norms and renormalisation
// (log-scale bookkeeping of the boundary MPSs), element-type conversion, the
// Philox4x64-10 generator (Salmon et al., SC'11) for random initial guesses and
// for the sampler's draws, the draw itself, and output bookkeeping.
#include "kernels.hpp"

#include <cmath>

namespace tnk {
namespace {

constexpr int NT = 256;

__device__ inline double2 ldc(const void *p, int esz, int64_t i) {
    if (esz == 16) return reinterpret_cast<const double2 *>(p)[i];
    const float2 f = reinterpret_cast<const float2 *>(p)[i];
    return make_double2(f.x, f.y);
}
__device__ inline void stc(void *p, int esz, int64_t i, double2 v) {
    if (esz == 16) reinterpret_cast<double2 *>(p)[i] = v;
    else reinterpret_cast<float2 *>(p)[i] = make_float2((float)v.x, (float)v.y);
}

__device__ inline double wsum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sum over the block in a fixed order (deterministic).
__device__ inline double bsum(double v) {
    __shared__ double red[NT / 64];
    v = wsum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int i = 0; i < NT / 64; ++i) s += red[i];
    __syncthreads();
    return s;
}

__global__ void __launch_bounds__(NT) k_norm2_part(const void *x, int esz, int64_t n, int64_t bs,
                                                  int P, double *partial) {
    const int b = blockIdx.y;
    const char *xb = reinterpret_cast<const char *>(x) + (int64_t)b * bs * esz;
    double s = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)P * NT) {
        const double2 v = ldc(xb, esz, i);
        s += v.x * v.x + v.y * v.y;
    }
    s = bsum(s);
    if (threadIdx.x == 0) partial[(int64_t)b * P + blockIdx.x] = s;
}

__global__ void k_sum_parts(const double *partial, int P, int batch, double *out) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    double s = 0.0;
    for (int i = 0; i < P; ++i) s += partial[(int64_t)b * P + i];
    out[b] = s;
}

__global__ void __launch_bounds__(NT) k_normalise(void *x, int esz, int64_t n, int64_t bs,
                                                 const double *norm2, double *logscale, int acc,
                                                 int *flags) {
    const int b = blockIdx.y;
    const double q = norm2[b];
    const bool bad = !(q > 0.0) || !isfinite(q);
    const double f = bad ? 1.0 : 1.0 / sqrt(q);
    char *xb = reinterpret_cast<char *>(x) + (int64_t)b * bs * esz;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        double2 v = ldc(xb, esz, i);
        v.x *= f; v.y *= f;
        stc(xb, esz, i, v);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (logscale) logscale[b] = (acc ? logscale[b] : 0.0) + (bad ? 0.0 : 0.5 * log(q));
        if (bad && flags) flags[b] |= 1;
    }
}

__global__ void __launch_bounds__(NT) k_convert(const void *src, int se, void *dst, int de, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        stc(dst, de, i, ldc(src, se, i));
}

__global__ void __launch_bounds__(NT) k_fill(void *x, int esz, int64_t n, double re, double im) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        stc(x, esz, i, make_double2(re, im));
}

// x[b] = n x n identity, `batch` matrices back to back.
__global__ void __launch_bounds__(NT) k_eye(void *x, int esz, int n, int64_t total) {
    const int64_t nn = (int64_t)n * n;
    for (int64_t e = (int64_t)blockIdx.x * NT + threadIdx.x; e < total; e += (int64_t)gridDim.x * NT) {
        const int64_t r = e % nn;
        stc(x, esz, e, make_double2(r / n == r % n ? 1.0 : 0.0, 0.0));
    }
}

// Philox4x64-10: ten rounds of two 64x64 -> 128-bit products with a Weyl key schedule.
__device__ inline void philox4x64_10(uint64_t c[4], uint64_t k0, uint64_t k1) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
    const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t hi0 = __umul64hi(M0, c[0]), lo0 = M0 * c[0];
        const uint64_t hi1 = __umul64hi(M1, c[2]), lo1 = M1 * c[2];
        const uint64_t n0 = hi1 ^ c[1] ^ k0;
        const uint64_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0; c[1] = lo1; c[2] = n2; c[3] = lo0;
        k0 += W0; k1 += W1;
    }
}
__device__ inline double u53(uint64_t w) { return (double)(w >> 11) * 0x1p-53; }

__global__ void __launch_bounds__(NT) k_init(void *out, int esz, int64_t n, int64_t bs, uint64_t seed,
                                            uint64_t tag, uint64_t row, uint64_t site,
                                            const uint64_t *sample) {
    const int b = blockIdx.y;
    const uint64_t smp = sample ? sample[b] : 0ull;
    char *ob = reinterpret_cast<char *>(out) + (int64_t)b * bs * esz;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) {
        uint64_t c[4] = {(uint64_t)i, site, row, smp};
        philox4x64_10(c, seed, tag);
        stc(ob, esz, i, make_double2(2.0 * u53(c[0]) - 1.0, 2.0 * u53(c[1]) - 1.0));
    }
}

__global__ void __launch_bounds__(NT) k_dot_part(const void *x, const void *y, int esz, int64_t n,
                                                int64_t bs, int P, double *partial, const int *mask,
                                                int mask_skip) {
    const int b = blockIdx.y;
    if (mask && mask[b] == mask_skip) return;
    const char *xb = reinterpret_cast<const char *>(x) + (int64_t)b * bs * esz;
    const char *yb = reinterpret_cast<const char *>(y) + (int64_t)b * bs * esz;
    double sr = 0.0, si = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)P * NT) {
        const double2 a = ldc(xb, esz, i), c = ldc(yb, esz, i);
        sr += a.x * c.x - a.y * c.y;
        si += a.x * c.y + a.y * c.x;
    }
    sr = bsum(sr);
    si = bsum(si);
    if (threadIdx.x == 0) {
        partial[((int64_t)b * P + blockIdx.x) * 2] = sr;
        partial[((int64_t)b * P + blockIdx.x) * 2 + 1] = si;
    }
}

__global__ void k_sum_parts2(const double *partial, int P, int batch, double *out, const int *mask,
                             int mask_skip) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    if (mask && mask[b] == mask_skip) return;
    double sr = 0.0, si = 0.0;
    for (int i = 0; i < P; ++i) {
        sr += partial[((int64_t)b * P + i) * 2];
        si += partial[((int64_t)b * P + i) * 2 + 1];
    }
    out[2 * b] = sr;
    out[2 * b + 1] = si;
}

__global__ void k_draw(DrawArgs a) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= a.batch) return;
    const double r0 = a.pt0[2 * b], r1 = a.pt1[2 * b];
    const double p0 = r0 > 0.0 ? r0 : 0.0;
    const double p1 = r1 > 0.0 ? r1 : 0.0;
    const double tot = p0 + p1;
    int x = 0;
    double lp = 0.0;
    if (!(tot > 0.0) || !isfinite(tot)) {
        a.flags[b] |= 2;
    } else {
        const double P0 = p0 / tot;
        double u;
        if (a.uniforms) {
            u = a.uniforms[(a.u_row0 + b) * (int64_t)a.n_qubits + a.qubit];
        } else {
            uint64_t c[4] = {(uint64_t)a.qubit, a.sample_index[b], 0ull, 0ull};
            philox4x64_10(c, a.seed, 3ull);
            u = u53(c[0]);
        }
        x = (u < P0) ? 0 : 1;
        lp = log(x == 0 ? P0 : p1 / tot);
    }
    a.log_q[b] += lp;
    if (a.log_cond) a.log_cond[(a.bits_row0 + b) * (int64_t)a.n_qubits + a.qubit] = lp;
    a.bits[(a.bits_row0 + b) * (int64_t)a.n_qubits + a.qubit] = (uint8_t)x;
    a.xsel[b] = x;
}

__global__ void k_select_offsets(const int *xsel, int batch, int64_t base, int64_t stride, int64_t *dst) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b < batch) dst[b] = base + (int64_t)xsel[b] * stride;
}

__global__ void __launch_bounds__(NT) k_select_copy(const void *x, int esz, int64_t n, int64_t ss,
                                                   int64_t bs, const int *sel, void *out, int64_t obs) {
    const int b = blockIdx.y;
    const int64_t src = (int64_t)b * bs + (int64_t)sel[b] * ss;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        stc(out, esz, (int64_t)b * obs + i, ldc(x, esz, src + i));
}

__global__ void __launch_bounds__(NT) k_select2(const void *x0, const void *x1, int esz, int64_t n, int64_t bs,
                                               const int *sel, void *out) {
    const int b = blockIdx.y;
    const void *x = sel[b] ? x1 : x0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        stc(out, esz, (int64_t)b * bs + i, ldc(x, esz, (int64_t)b * bs + i));
}

__global__ void __launch_bounds__(NT) k_fill_f64(double *x, int64_t n, double v) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) x[i] = v;
}

__global__ void __launch_bounds__(NT) k_fill_i32(int *x, int64_t n, int v) {
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT) x[i] = v;
}

__global__ void k_env_rho(const double *d, double *out) {
    const int i = threadIdx.x;  // 4 entries
    const double tr = d[0] + d[6], ti = d[1] + d[7];
    const double den = tr * tr + ti * ti;
    if (i < 4) {
        const double a = d[2 * i], b = d[2 * i + 1];
        out[2 * i] = (a * tr + b * ti) / den;
        out[2 * i + 1] = (b * tr - a * ti) / den;
    }
}

__global__ void k_env_p2(const double *d, double *p2, double *zz) {
    if (threadIdx.x != 0) return;
    const double P0 = d[0], P1 = d[2], P2 = d[4], P3 = d[6];
    const double S = P0 + P1 + P2 + P3;
    if (p2) { p2[0] = P0 / S; p2[1] = P1 / S; p2[2] = P2 / S; p2[3] = P3 / S; }
    if (zz) *zz = (P0 - P1 - P2 + P3) / S;
}

__global__ void k_logp(const double *amp, const double *mlog, int batch, double *log_p, double *arg) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= batch) return;
    const double a = hypot(amp[2 * b], amp[2 * b + 1]);
    log_p[b] = a > 0.0 ? 2.0 * (mlog[b] + log(a)) : -INFINITY;
    if (arg) arg[b] = atan2(amp[2 * b + 1], amp[2 * b]);
}

__global__ void k_marginal_rest(const double *tot, const double *lnr, const double *pt0, double *pt1, int batch,
                                double thr, int *need) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= batch) return;
    const double f = exp(lnr[z]);
    const double tr = f * tot[2 * z], ti = f * tot[2 * z + 1];
    const double dr = tr - pt0[2 * z];
    pt1[2 * z] = dr;
    pt1[2 * z + 1] = ti - pt0[2 * z + 1];
    // a difference below thr of the total is not trusted (not even its sign):
    // that sample's projection is contracted directly
    need[z] = (dr > thr * tr) ? 0 : 1;
}

// out[z] = 1 for the samples that drew the bit `other` and whose projection on
// it was not contracted before the draw (need[z] == 0), else 0.
__global__ void k_other_mask(const int *xs, const int *need, int other, int batch, int *out) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= batch) return;
    out[z] = (xs[z] == other && !need[z]) ? 1 : 0;
}

// For the samples that drew `other`: replace the log-conditional the draw
// used (from P~(other) = pt_used) by the one from the directly contracted
// P~(other) = pt_direct, with the favoured bit's P~ = pt_f.
__global__ void k_fix_other(const double *pt_f, const double *pt_used, const double *pt_direct, const int *xs,
                            int other, int batch, double *log_q, double *log_cond, int64_t row0, int n_qubits,
                            int qubit, int *flags) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= batch || xs[z] != other) return;
    const double pf = fmax(pt_f[2 * z], 0.0);
    const double pu = fmax(pt_used[2 * z], 0.0);
    const double pd = pt_direct[2 * z];
    if (!(pd > 0.0) || !isfinite(pd)) {
        flags[z] |= 2;
        return;
    }
    const double lnew = log(pd / (pf + pd));
    log_q[z] += lnew - log(pu / (pf + pu));
    if (log_cond) log_cond[(row0 + z) * (int64_t)n_qubits + qubit] = lnew;
}

// Per-sample bond of the amplitude boundary: the largest kept value over the cuts.
__global__ void k_chi_used(const int *k, int cuts, int batch, int constant, int *out, int64_t stride) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= batch) return;
    int v = constant;
    if (k && cuts > 0) {
        v = 0;
        for (int c = 0; c < cuts; ++c) v = max(v, k[(int64_t)c * batch + z]);
    }
    out[(int64_t)z * stride] = v;
}

// xs[z] = bits[(row0 + z) * n_qubits + qubit]: the given bit of every sample of
// a wave, as the selector of the projected row tensor.
__global__ void k_bits_select(const uint8_t *bits, int64_t n_qubits, int64_t row0, int qubit, int batch, int *xs) {
    const int z = blockIdx.x * blockDim.x + threadIdx.x;
    if (z >= batch) return;
    xs[z] = bits[(row0 + z) * n_qubits + qubit] ? 1 : 0;
}

// Sample-quality metrics over n samples, in three passes over P blocks of SN
// threads with partial results in a workspace, fixed reduction order.
// w_i = exp(lw_i - max lw), lw = log p - log q:
// out[0] = log((1/n) sum p/q), out[1] = (1/n) sum (log q - log p + log Z),
// out[2] = (sum w)^2 / sum w^2; z_is[q] = sum_i w_i (1 - 2 x_iq) / sum_i w_i.
// Block b covers samples [b c, min(n, (b+1) c)), c = ceil(n / P).
constexpr int SN = 256;
constexpr int SW = 1024;  // weights staged in LDS per chunk (z_is pass)
__device__ double block_sum(double v, double *red) {
    red[threadIdx.x] = v;
    __syncthreads();
    for (int h = SN / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    const double r = red[0];
    __syncthreads();
    return r;
}

__device__ inline void stats_range(int64_t n, int P, int64_t &beg, int64_t &end) {
    const int64_t c = (n + P - 1) / P;
    beg = (int64_t)blockIdx.x * c;
    end = beg + c < n ? beg + c : n;
}

__global__ void __launch_bounds__(SN) k_stats_max(const double *lq, const double *lp, int64_t n, int P,
                                                  double *pmax) {
    __shared__ double red[SN];
    int64_t beg, end;
    stats_range(n, P, beg, end);
    double mx = -INFINITY;
    for (int64_t i = beg + threadIdx.x; i < end; i += SN) mx = fmax(mx, lp[i] - lq[i]);
    red[threadIdx.x] = mx;
    __syncthreads();
    for (int h = SN / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + h]);
        __syncthreads();
    }
    if (threadIdx.x == 0) pmax[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(SN) k_stats_sums(const double *lq, const double *lp, int64_t n, double logZ,
                                                   const uint8_t *bits, int64_t nq, int P, const double *pmax,
                                                   double *psum, double *pz) {
    __shared__ double red[SN];
    __shared__ double wl[SW];
    double top = -INFINITY;
    for (int b = 0; b < P; ++b) top = fmax(top, pmax[b]);
    int64_t beg, end;
    stats_range(n, P, beg, end);
    double s1 = 0.0, s2 = 0.0, kl = 0.0;
    for (int64_t i = beg + threadIdx.x; i < end; i += SN) {
        const double w = exp(lp[i] - lq[i] - top);
        s1 += w;
        s2 += w * w;
        kl += lq[i] - lp[i] + logZ;
    }
    s1 = block_sum(s1, red);
    s2 = block_sum(s2, red);
    kl = block_sum(kl, red);
    if (threadIdx.x == 0) {
        psum[3 * blockIdx.x] = s1;
        psum[3 * blockIdx.x + 1] = s2;
        psum[3 * blockIdx.x + 2] = kl;
    }
    if (!pz) return;
    double *zb = pz + (int64_t)blockIdx.x * nq;
    for (int64_t q = threadIdx.x; q < nq; q += SN) zb[q] = 0.0;  // each (block, q) is owned by one thread
    for (int64_t c0 = beg; c0 < end; c0 += SW) {
        const int len = (int)(end - c0 < SW ? end - c0 : SW);
        __syncthreads();
        for (int i = threadIdx.x; i < len; i += SN) wl[i] = exp(lp[c0 + i] - lq[c0 + i] - top);
        __syncthreads();
        for (int64_t q = threadIdx.x; q < nq; q += SN) {
            double acc = 0.0;
            for (int i = 0; i < len; ++i) acc += bits[(c0 + i) * nq + q] ? -wl[i] : wl[i];
            zb[q] += acc;
        }
    }
}

__global__ void __launch_bounds__(SN) k_stats_final(const double *psum, const double *pz, int P, int64_t n,
                                                    int64_t nq, const double *pmax, double *out, double *z_is) {
    __shared__ double s1s;
    if (threadIdx.x == 0) {
        double top = -INFINITY, s1 = 0.0, s2 = 0.0, kl = 0.0;
        for (int b = 0; b < P; ++b) {
            top = fmax(top, pmax[b]);
            s1 += psum[3 * b];
            s2 += psum[3 * b + 1];
            kl += psum[3 * b + 2];
        }
        out[0] = top + log(s1 / (double)n);
        out[1] = kl / (double)n;
        out[2] = s1 * s1 / s2;
        s1s = s1;
    }
    __syncthreads();
    if (!z_is) return;
    for (int64_t q = threadIdx.x; q < nq; q += SN) {
        double acc = 0.0;
        for (int b = 0; b < P; ++b) acc += pz[(int64_t)b * nq + q];
        z_is[q] = acc / s1s;
    }
}

// Fingerprint of raw tensor bytes: acc += sum_i mix(word_i, salt + i), with
// the splitmix64 finaliser as the mixer (sum modulo 2^64).  Words are 8 bytes.
__device__ inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void __launch_bounds__(NT) k_fingerprint(FingerprintSet f, unsigned long long *acc) {
    const int t = blockIdx.y;
    const uint64_t *x = reinterpret_cast<const uint64_t *>(f.ptr[t]);
    const int64_t n = f.words[t];
    const uint64_t salt = f.salt[t];
    uint64_t h = 0;
    for (int64_t i = (int64_t)blockIdx.x * NT + threadIdx.x; i < n; i += (int64_t)gridDim.x * NT)
        h += mix64(x[i] ^ mix64(salt + (uint64_t)i * 0x9E3779B97F4A7C15ull));
    for (int o = 32; o > 0; o >>= 1) h += __shfl_xor(h, o);
    if ((threadIdx.x & 63) == 0 && h) atomicAdd(acc, (unsigned long long)h);
}

int grid_for(int64_t n) {
    int64_t g = (n + NT - 1) / NT;
    if (g > 4096) g = 4096;
    if (g < 1) g = 1;
    return (int)g;
}

}  // namespace

int reduce_partial_count(int64_t n) {
    int64_t p = (n + 16383) / 16384;
    if (p < 1) p = 1;
    if (p > 256) p = 256;
    return (int)p;
}

hipError_t launch_norm2(const void *x, int esz, int64_t n, int batch, int64_t bs, double *partial,
                        double *out, hipStream_t s) {
    const int P = reduce_partial_count(n);
    hipLaunchKernelGGL(k_norm2_part, dim3(P, batch), dim3(NT), 0, s, x, esz, n, bs, P, partial);
    hipLaunchKernelGGL(k_sum_parts, dim3((batch + 63) / 64), dim3(64), 0, s, partial, P, batch, out);
    return hipGetLastError();
}

hipError_t launch_normalise(void *x, int esz, int64_t n, int batch, int64_t bs, const double *norm2,
                            double *logscale, int acc, int *flags, hipStream_t s) {
    int g = grid_for(n);
    if (g > 512) g = 512;
    hipLaunchKernelGGL(k_normalise, dim3(g, batch), dim3(NT), 0, s, x, esz, n, bs, norm2, logscale, acc, flags);
    return hipGetLastError();
}

hipError_t launch_convert(const void *src, int se, void *dst, int de, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_convert, dim3(grid_for(n)), dim3(NT), 0, s, src, se, dst, de, n);
    return hipGetLastError();
}

hipError_t launch_fill(void *x, int esz, int64_t n, double re, double im, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(NT), 0, s, x, esz, n, re, im);
    return hipGetLastError();
}

hipError_t launch_eye(void *x, int esz, int n, int batch, hipStream_t s) {
    const int64_t total = (int64_t)n * n * batch;
    if (total <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_eye, dim3(grid_for(total)), dim3(NT), 0, s, x, esz, n, total);
    return hipGetLastError();
}

hipError_t launch_init_tensor(void *out, int esz, int64_t n, int batch, int64_t bs, uint64_t seed,
                              uint64_t tag, uint64_t row, uint64_t site, const uint64_t *sample,
                              hipStream_t s) {
    if (n <= 0 || batch <= 0) return hipSuccess;
    int g = grid_for(n);
    if (g > 512) g = 512;
    hipLaunchKernelGGL(k_init, dim3(g, batch), dim3(NT), 0, s, out, esz, n, bs, seed, tag, row, site, sample);
    return hipGetLastError();
}

hipError_t launch_dot(const void *x, const void *y, int esz, int64_t n, int batch, int64_t bs,
                      double *partial, double *out, hipStream_t s, const int *mask, int mask_skip) {
    const int P = reduce_partial_count(n);
    hipLaunchKernelGGL(k_dot_part, dim3(P, batch), dim3(NT), 0, s, x, y, esz, n, bs, P, partial, mask,
                       mask_skip);
    hipLaunchKernelGGL(k_sum_parts2, dim3((batch + 63) / 64), dim3(64), 0, s, partial, P, batch, out, mask,
                       mask_skip);
    return hipGetLastError();
}

hipError_t launch_draw(const DrawArgs &a, hipStream_t s) {
    hipLaunchKernelGGL(k_draw, dim3((a.batch + 63) / 64), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_select_offsets(const int *xsel, int batch, int64_t base, int64_t stride, int64_t *dst,
                                 hipStream_t s) {
    hipLaunchKernelGGL(k_select_offsets, dim3((batch + 63) / 64), dim3(64), 0, s, xsel, batch, base, stride, dst);
    return hipGetLastError();
}

hipError_t launch_select_copy(const void *x, int esz, int64_t n, int64_t ss, int64_t bs, const int *sel,
                              int batch, void *out, int64_t obs, hipStream_t s) {
    int g = grid_for(n);
    if (g > 512) g = 512;
    hipLaunchKernelGGL(k_select_copy, dim3(g, batch), dim3(NT), 0, s, x, esz, n, ss, bs, sel, out, obs);
    return hipGetLastError();
}

hipError_t launch_select2(const void *x0, const void *x1, int esz, int64_t n, int64_t bs, const int *sel,
                          int batch, void *out, hipStream_t s) {
    int g = grid_for(n);
    if (g > 512) g = 512;
    hipLaunchKernelGGL(k_select2, dim3(g, batch), dim3(NT), 0, s, x0, x1, esz, n, bs, sel, out);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *x, int64_t n, double v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(n)), dim3(NT), 0, s, x, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_i32(int *x, int64_t n, int v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(n)), dim3(NT), 0, s, x, n, v);
    return hipGetLastError();
}

hipError_t launch_env_rho(const double *dots, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_env_rho, dim3(1), dim3(64), 0, s, dots, out);
    return hipGetLastError();
}

hipError_t launch_env_p2(const double *dots, double *p2, double *zz, hipStream_t s) {
    hipLaunchKernelGGL(k_env_p2, dim3(1), dim3(64), 0, s, dots, p2, zz);
    return hipGetLastError();
}

hipError_t launch_bits_select(const uint8_t *bits, int64_t n_qubits, int64_t row0, int qubit, int batch, int *xs,
                              hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_bits_select, dim3((batch + 63) / 64), dim3(64), 0, s, bits, n_qubits, row0, qubit, batch, xs);
    return hipGetLastError();
}

int stats_blocks(int64_t n) {
    int64_t p = (n + 1023) / 1024;
    if (p < 1) p = 1;
    if (p > STATS_BLOCKS_MAX) p = STATS_BLOCKS_MAX;
    return (int)p;
}

size_t stats_workspace_bytes(int64_t n, int64_t n_qubits, bool with_z) {
    const int64_t P = stats_blocks(n);
    return (size_t)(4 * P + (with_z ? P * n_qubits : 0)) * sizeof(double);
}

hipError_t launch_sample_stats(const double *log_q, const double *log_p, int64_t n, double log_Z,
                               const uint8_t *bits, int64_t n_qubits, double *out, double *z_is, void *workspace,
                               hipStream_t s) {
    if (n <= 0 || !workspace) return hipErrorInvalidValue;
    const int P = stats_blocks(n);
    double *pmax = static_cast<double *>(workspace);
    double *psum = pmax + P;
    double *pz = z_is ? psum + 3 * P : nullptr;
    hipLaunchKernelGGL(k_stats_max, dim3(P), dim3(SN), 0, s, log_q, log_p, n, P, pmax);
    hipLaunchKernelGGL(k_stats_sums, dim3(P), dim3(SN), 0, s, log_q, log_p, n, log_Z, z_is ? bits : nullptr,
                       n_qubits, P, pmax, psum, pz);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(SN), 0, s, psum, pz, P, n, n_qubits, pmax, out, z_is);
    return hipGetLastError();
}

hipError_t launch_marginal_rest(const double *tot, const double *lnr, const double *pt0, double *pt1, int batch,
                                double thr, int *need, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_marginal_rest, dim3((batch + 63) / 64), dim3(64), 0, s, tot, lnr, pt0, pt1, batch, thr,
                       need);
    return hipGetLastError();
}

hipError_t launch_other_mask(const int *xs, const int *need, int other, int batch, int *out, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_other_mask, dim3((batch + 63) / 64), dim3(64), 0, s, xs, need, other, batch, out);
    return hipGetLastError();
}

hipError_t launch_fix_other(const double *pt_f, const double *pt_used, const double *pt_direct, const int *xs,
                            int other, int batch, double *log_q, double *log_cond, int64_t row0, int n_qubits,
                            int qubit, int *flags, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fix_other, dim3((batch + 63) / 64), dim3(64), 0, s, pt_f, pt_used, pt_direct, xs, other,
                       batch, log_q, log_cond, row0, n_qubits, qubit, flags);
    return hipGetLastError();
}

hipError_t launch_chi_used(const int *k, int cuts, int batch, int constant, int *out, int64_t stride,
                           hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_chi_used, dim3((batch + 63) / 64), dim3(64), 0, s, k, cuts, batch, constant, out, stride);
    return hipGetLastError();
}

hipError_t launch_logp(const double *amp, const double *mlog, int batch, double *log_p, double *arg,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_logp, dim3((batch + 63) / 64), dim3(64), 0, s, amp, mlog, batch, log_p, arg);
    return hipGetLastError();
}

hipError_t launch_fingerprint(const FingerprintSet &f, unsigned long long *acc, hipStream_t s) {
    if (f.count <= 0) return hipSuccess;
    int64_t mx = 1;
    for (int i = 0; i < f.count; ++i) mx = f.words[i] > mx ? f.words[i] : mx;
    int g = grid_for(mx);
    if (g > 64) g = 64;
    hipLaunchKernelGGL(k_fingerprint, dim3(g, f.count), dim3(NT), 0, s, f, acc);
    return hipGetLastError();
}

}  // namespace tnk
