// Small kernels of the simple-update gate step (Appendix, "Applying Gates to a
// Tensor Network State"): square roots of the BP messages, the balanced split
// of the truncated SVD between the two sites, and the table-driven block copies
// that gather the tensors of a batch of gates and scatter the results.
#include "kernels.hpp"

#include <algorithm>

namespace tnk {
namespace {

// One workgroup of 256 threads per matrix: the singular values from the
// rows of SV, then every element of both outputs.
__global__ void __launch_bounds__(256) k_msg_roots(const double2 *U, const double2 *SV, int n, double2 *Sq,
                                                   double2 *Sp) {
    __shared__ double sig[64];
    const int b = blockIdx.x, t = threadIdx.x;
    const int64_t off = (int64_t)b * n * n;
    if (t < n) {
        double v = 0.0;
        for (int l = 0; l < n; ++l) {
            const double2 x = SV[off + (int64_t)t * n + l];
            v += x.x * x.x + x.y * x.y;
        }
        sig[t] = sqrt(v);
    }
    __syncthreads();
    for (int e = t; e < n * n; e += 256) {
        const int i = e / n, j = e % n;
        double2 q = make_double2(0.0, 0.0), p = make_double2(0.0, 0.0);
        for (int c = 0; c < n; ++c) {
            const double s = sig[c];
            if (!(s > 0.0)) continue;
            const double2 u = U[off + (int64_t)i * n + c], v = SV[off + (int64_t)c * n + j];
            const double2 uv = make_double2(u.x * v.x - u.y * v.y, u.x * v.y + u.y * v.x);
            const double fq = 1.0 / sqrt(s), fp = fq / s;
            q.x += fq * uv.x; q.y += fq * uv.y;
            p.x += fp * uv.x; p.y += fp * uv.y;
        }
        Sq[off + e] = q;
        Sp[off + e] = p;
    }
}

__global__ void __launch_bounds__(256) k_split_sqrt(double2 *U, double2 *SV, int n) {
    __shared__ double rs[256];
    const int b = blockIdx.x, t = threadIdx.x;
    const int64_t off = (int64_t)b * n * n;
    if (t < n) {
        double v = 0.0;
        for (int l = 0; l < n; ++l) {
            const double2 x = SV[off + (int64_t)t * n + l];
            v += x.x * x.x + x.y * x.y;
        }
        rs[t] = sqrt(sqrt(v));  // sigma^{1/2}
    }
    __syncthreads();
    for (int e = t; e < n * n; e += 256) {
        const int i = e / n, j = e % n;
        const double su = rs[j], sv = rs[i];
        double2 u = U[off + e], w = SV[off + e];
        u.x *= su; u.y *= su;  // U[i][j]: column j
        if (sv > 0.0) { w.x /= sv; w.y /= sv; }  // SV[i][j]: row i
        U[off + e] = u;
        SV[off + e] = w;
    }
}

// Workgroup (x, y) copies the elements y, y + Y, ... (in units of 256) of
// table entry x: dst[e] = src[(e / cols) * src_ld + e % cols].
__global__ void __launch_bounds__(256) k_copy_blocks(const CopyBlock *tab) {
    const CopyBlock b = tab[blockIdx.x];
    const double2 *src = static_cast<const double2 *>(b.src);
    double2 *dst = static_cast<double2 *>(b.dst);
    const int64_t total = b.rows * b.cols;
    for (int64_t e = (int64_t)blockIdx.y * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.y * 256) {
        const int64_t r = e / b.cols, c = e - r * b.cols;
        dst[e] = src[r * b.src_ld + c];
    }
}

}  // namespace

hipError_t launch_copy_blocks(const CopyBlock *tab, int n, int64_t max_elems, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    if (!tab || max_elems < 0) return hipErrorInvalidValue;
    const int64_t y = std::min<int64_t>(std::max<int64_t>((max_elems + 4095) / 4096, 1), 256);
    hipLaunchKernelGGL(k_copy_blocks, dim3(n, (unsigned)y), dim3(256), 0, s, tab);
    return hipGetLastError();
}

hipError_t launch_msg_roots(const double *U, const double *SV, int n, int batch, double *Sq, double *Sp,
                            hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    if (n < 1 || n > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_msg_roots, dim3(batch), dim3(256), 0, s, reinterpret_cast<const double2 *>(U),
                       reinterpret_cast<const double2 *>(SV), n, reinterpret_cast<double2 *>(Sq),
                       reinterpret_cast<double2 *>(Sp));
    return hipGetLastError();
}

hipError_t launch_split_sqrt(double *U, double *SV, int n, int batch, hipStream_t s) {
    if (batch <= 0) return hipSuccess;
    if (n < 1 || n > 256) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_split_sqrt, dim3(batch), dim3(256), 0, s, reinterpret_cast<double2 *>(U),
                       reinterpret_cast<double2 *>(SV), n);
    return hipGetLastError();
}

}  // namespace tnk
