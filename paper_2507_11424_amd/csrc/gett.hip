// Complex tensor contraction engine on CDNA4 matrix cores.
//
// Every contraction of the boundary-MPS fit and of the sampler (products of
// boundary MPS, row tensors, their conjugates and environments) is a batched
// complex GEMM over gathered indices (see GettArgs).  Complex products use the
// 4M form on real MFMA:
//   Re C += Re A Re B - Im A Im B,   Im C += Re A Im B + Im A Re B,
// with A and B tiles staged through LDS as planar (re, im) slabs.
//
// Precisions:
//   FP64   : complex128 storage, v_mfma_f64_16x16x4_f64;
//   FP32   : complex64 storage, v_mfma_f32_16x16x4_f32;
//   BF16X3 : complex64 storage; each FP32 value x is split at LDS-staging time
//            into bf16 parts x = h + l (+ residual), and a product a*b is
//            formed as ah*bh + ah*bl + al*bh with v_mfma_f32_16x16x32_bf16,
//            accumulated in FP32;
//   BF16X6 : three parts x = h + m + l, products hh + hm + mh + hl + lh + mm.
#include "kernels.hpp"

namespace tnk {
namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef short v8s __attribute__((ext_vector_type(8)));
typedef unsigned int v4u __attribute__((ext_vector_type(4)));

template <typename T> struct Tr;
// Accumulator layout of the 16x16 MFMA forms: lane l, register r holds row
//   FP64 (16x16x4 f64):      4 r + l / 16
//   FP32 / BF16 16x16 forms: 4 (l / 16) + r
// and column l % 16 in both.
template <> struct Tr<double> {
    using C2 = double2;
    using Acc = v4d;
    __device__ static inline int row(int lane, int r) { return 4 * r + (lane >> 4); }
    __device__ static inline Acc mma(double a, double b, Acc c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
};
template <> struct Tr<float> {
    using C2 = float2;
    using Acc = v4f;
    __device__ static inline int row(int lane, int r) { return 4 * (lane >> 4) + r; }
    __device__ static inline Acc mma(float a, float b, Acc c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
};

__device__ inline int xcd_remap(int t, int ntiles) {
    // workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
    // contiguous range of tiles so that tiles sharing an A panel share an L2
    if ((ntiles & 7) != 0) return t;
    return (t & 7) * (ntiles >> 3) + (t >> 3);
}

// Tile skip of a masked launch (see GettArgs::mask); block-uniform.
__device__ inline bool gett_skip(const GettArgs &p, int b, int m0, int n0) {
    if (!p.mask) return false;
    const int c = p.mask_mode == 1 ? b : (p.mask_mode == 2 ? m0 : n0);
    return p.mask[c / p.mask_div] == p.mask_skip;
}

// --------------------------------------------------------------------------
// Operand staging shared by the kernels.
//
// Operands are read with raw buffer loads: the resource covers the operand's
// window for the batch item, and an offset of 2^31 (beyond every window) makes
// the hardware return zero, so the tile's ragged edges need no branches and all
// loads of a stage issue back to back.  k offsets are affine (k * ks, kept in
// registers) or come from the k table, staged into LDS once per block.
constexpr uint32_t OOB = 0x80000000u;
constexpr bool GAUSS3M = true;  // 64x64 and 64x16 FP64 / FP32 tiles; 128x64 keeps 4M (3M would spill)

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
    // the base is the same for the whole workgroup (batch item); say so, so
    // that the resource lives in scalar registers
    const uint64_t a = reinterpret_cast<uint64_t>(p);
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)a);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(a >> 32));
    void *u = reinterpret_cast<void *>(((uint64_t)hi << 32) | lo);
    // dword 3 of a gfx9 buffer resource: 32-bit data format, no swizzle
    return __builtin_amdgcn_make_buffer_rsrc(u, (short)0, (int)__builtin_amdgcn_readfirstlane(bytes), 0x00020000);
}
template <typename C2> __device__ inline C2 bload(__amdgpu_buffer_rsrc_t r, uint32_t off);
template <> __device__ inline double2 bload<double2>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(double2, __builtin_amdgcn_raw_buffer_load_b128(r, (int)off, 0, 0));
}
template <> __device__ inline float2 bload<float2>(__amdgpu_buffer_rsrc_t r, uint32_t off) {
    return __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, 0, 0));
}

// Per-thread view of one operand tile: L elements at (row r[i], k index k[i])
// inside the tile; row offsets resolved once per block.
template <int L>
struct Stager {
    int ro[L];   // element offset of the row (m or n), -1 outside the matrix
    int kk[L];   // k index inside the tile
    const int *kt;  // LDS k table (block's K slice) or null when affine
    int ks, kbeg, kend;
    __device__ inline uint32_t off(int i, int k0, int esz) const {
        const int k = k0 + kk[i];
        const bool ok = ro[i] >= 0 && k < kend;
        const int kc = k < kend ? k : kend - 1;
        const int ko = kt ? kt[kc - kbeg] : kc * ks;
        return ok ? (uint32_t)(ro[i] + ko) * (uint32_t)esz : OOB;
    }
};

// Copies the block's K slice of a k table into LDS.
__device__ inline void stage_ktab(int *dst, const int32_t *tab, int kbeg, int klen, int tid, int nt) {
    for (int k = tid; k < klen; k += nt) dst[k] = tab[kbeg + k];
}

// --------------------------------------------------------------------------
// FP64 / FP32: one MFMA 16x16x4 per real product; 4 per complex product (4M)
// or 3 with the Gauss form (3M): aR bR, aI bI and (aR + aI)(bR + bI), the
// sums formed in registers after the LDS reads.  3M saves a quarter of the
// MFMA work; its imaginary part, P3 - P1 - P2, carries about twice the
// rounding error of 4M relative to sum |a||b|.
// Two LDS stages: the tile for step k+1 is loaded from HBM into registers while
// step k computes, then stored to the other stage; one barrier per step.
template <typename T, int BM, int BN, int BK, int WGM, int WGN, bool G3>
__global__ void __launch_bounds__(64 * WGM * WGN, 2)
gett_mfma(GettArgs p) {
    using C2 = typename Tr<T>::C2;
    using Acc = typename Tr<T>::Acc;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int FM = WTM / 16, FN = WTN / 16;
    constexpr int LA = (BM * BK) / NT;
    constexpr int LB = (BK * BN) / NT;
    constexpr int PA = BM + 2, PB = BN + 2;
    constexpr int ESZ = (int)sizeof(C2);
    static_assert(LA >= 1 && LB >= 1 && NT % BK == 0 && NT >= BM && NT >= BN, "tile");
    __shared__ T sA[2][2][BK][PA];  // [stage][re/im][k][m]
    __shared__ T sB[2][2][BK][PB];
    extern __shared__ int ktab[];   // non-affine k tables of the block's K slice

    const int tid = threadIdx.x;
    const int tiles_n = (p.N + BN - 1) / BN;
    const int tiles_m = (p.M + BM - 1) / BM;
    // a masked launch keeps the dispatch order, which deals consecutive tiles
    // round-robin over the XCDs: with contiguous per-XCD ranges the tiles of
    // one sample would sit on one or two XCDs and the others would idle
    const int tile = p.mask ? (int)blockIdx.x : xcd_remap(blockIdx.x, tiles_m * tiles_n);
    const int m0 = (tile / tiles_n) * BM;
    const int n0 = (tile % tiles_n) * BN;
    const int kbeg = blockIdx.z * p.kchunk;
    const int kend = min(p.K, kbeg + p.kchunk);

    int am[LA], bn[LB];
    Stager<LA> sa;
    Stager<LB> sb;
#pragma unroll
    for (int i = 0; i < LA; ++i) {
        if (p.a_kfast) { sa.kk[i] = tid % BK; am[i] = tid / BK + (NT / BK) * i; }
        else           { am[i] = tid % BM; sa.kk[i] = tid / BM + (NT / BM) * i; }
        const int m = m0 + am[i];
        sa.ro[i] = (m < p.M) ? p.a_moff[m] : -1;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
        if (p.b_kfast) { sb.kk[i] = tid % BK; bn[i] = tid / BK + (NT / BK) * i; }
        else           { bn[i] = tid % BN; sb.kk[i] = tid / BN + (NT / BN) * i; }
        const int n = n0 + bn[i];
        sb.ro[i] = (n < p.N) ? p.b_noff[n] : -1;
    }
    sa.ks = p.a_ks; sb.ks = p.b_ks;
    sa.kbeg = sb.kbeg = kbeg;
    sa.kend = sb.kend = kend;
    sa.kt = p.a_kaff ? nullptr : ktab;
    sb.kt = p.b_kaff ? nullptr : ktab + (p.a_kaff ? 0 : p.kchunk);
    if (!p.a_kaff) stage_ktab(ktab, p.a_koff, kbeg, kend - kbeg, tid, NT);
    if (!p.b_kaff) stage_ktab(const_cast<int *>(sb.kt), p.b_koff, kbeg, kend - kbeg, tid, NT);

    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave / WGN, wn = wave % WGN;
    const T sgnA = p.conjA ? T(-1) : T(1);
    const T sgnB = p.conjB ? T(-1) : T(1);

    for (int b = blockIdx.y; b < p.batch; b += gridDim.y) {
        if (gett_skip(p, b, m0, n0)) continue;
        const __amdgpu_buffer_rsrc_t rA = make_rsrc(reinterpret_cast<const C2 *>(p.A) + p.a_boff[b], p.a_bytes);
        const __amdgpu_buffer_rsrc_t rB = make_rsrc(reinterpret_cast<const C2 *>(p.B) + p.b_boff[b], p.b_bytes);
        C2 *Cb = reinterpret_cast<C2 *>(p.C) + p.c_boff[b];

        // 4M: accR, accI.  3M (G3): accR = sum aR bR, accI = sum aI bI,
        // acc3 = sum (aR + aI)(bR + bI); Re = accR - accI, Im = acc3 - accR - accI.
        Acc accR[FM][FN], accI[FM][FN], acc3[G3 ? FM : 1][G3 ? FN : 1];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) { accR[i][j][r] = T(0); accI[i][j][r] = T(0); }
        if constexpr (G3) {
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j)
#pragma unroll
                    for (int r = 0; r < 4; ++r) acc3[i][j][r] = T(0);
        }

        C2 ra[LA], rb[LB];
        auto gload = [&](int k0) {
            uint32_t oa[LA], ob[LB];
#pragma unroll
            for (int i = 0; i < LA; ++i) oa[i] = sa.off(i, k0, ESZ);
#pragma unroll
            for (int i = 0; i < LB; ++i) ob[i] = sb.off(i, k0, ESZ);
#pragma unroll
            for (int i = 0; i < LA; ++i) ra[i] = bload<C2>(rA, oa[i]);
#pragma unroll
            for (int i = 0; i < LB; ++i) rb[i] = bload<C2>(rB, ob[i]);
        };
        auto lstore = [&](int st) {
#pragma unroll
            for (int i = 0; i < LA; ++i) {
                sA[st][0][sa.kk[i]][am[i]] = ra[i].x;
                sA[st][1][sa.kk[i]][am[i]] = sgnA * ra[i].y;
            }
#pragma unroll
            for (int i = 0; i < LB; ++i) {
                sB[st][0][sb.kk[i]][bn[i]] = rb[i].x;
                sB[st][1][sb.kk[i]][bn[i]] = sgnB * rb[i].y;
            }
        };
        // the previous batch item's last step may still read stage 0; the first
        // pass also publishes the LDS k tables
        __syncthreads();
        gload(kbeg);
        lstore(0);
        __syncthreads();
        int st = 0;
        for (int k0 = kbeg; k0 < kend; k0 += BK, st ^= 1) {
            const bool more = k0 + BK < kend;
            if (more) gload(k0 + BK);
#pragma unroll
            for (int kq = 0; kq < BK / 4; ++kq) {
                const int kr = kq * 4 + (lane >> 4);
                T arv[FM], aiv[FM], brv[FN], biv[FN];
#pragma unroll
                for (int i = 0; i < FM; ++i) {
                    const int mm = wm * WTM + i * 16 + (lane & 15);
                    arv[i] = sA[st][0][kr][mm];
                    aiv[i] = sA[st][1][kr][mm];
                }
#pragma unroll
                for (int j = 0; j < FN; ++j) {
                    const int nn = wn * WTN + j * 16 + (lane & 15);
                    brv[j] = sB[st][0][kr][nn];
                    biv[j] = sB[st][1][kr][nn];
                }
                if constexpr (G3) {
                    T asv[FM], bsv[FN];
#pragma unroll
                    for (int i = 0; i < FM; ++i) asv[i] = arv[i] + aiv[i];
#pragma unroll
                    for (int j = 0; j < FN; ++j) bsv[j] = brv[j] + biv[j];
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j) {
                            accR[i][j] = Tr<T>::mma(arv[i], brv[j], accR[i][j]);
                            accI[i][j] = Tr<T>::mma(aiv[i], biv[j], accI[i][j]);
                            acc3[i][j] = Tr<T>::mma(asv[i], bsv[j], acc3[i][j]);
                        }
                } else {
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j) {
                            accR[i][j] = Tr<T>::mma(arv[i], brv[j], accR[i][j]);
                            accI[i][j] = Tr<T>::mma(arv[i], biv[j], accI[i][j]);
                        }
#pragma unroll
                    for (int i = 0; i < FM; ++i)
#pragma unroll
                        for (int j = 0; j < FN; ++j) {
                            accR[i][j] = Tr<T>::mma(-aiv[i], biv[j], accR[i][j]);
                            accI[i][j] = Tr<T>::mma(aiv[i], brv[j], accI[i][j]);
                        }
                }
            }
            if (more) {
                // the other stage was last read in the previous step, before the
                // barrier that ended it
                lstore(st ^ 1);
                __syncthreads();
            }
        }
        // epilogue: see Tr<T>::row for the accumulator layout
        C2 *Pb = p.ksplit > 1
                     ? reinterpret_cast<C2 *>(p.part) + ((int64_t)blockIdx.z * p.batch + b) * (int64_t)p.M * p.N
                     : nullptr;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int n = n0 + wn * WTN + j * 16 + (lane & 15);
            if (n >= p.N) continue;
            const int64_t cn = Pb ? 0 : p.c_noff[n];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = m0 + wm * WTM + i * 16 + Tr<T>::row(lane, r);
                    if (m >= p.M) continue;
                    C2 v;
                    if constexpr (G3) {
                        v.x = accR[i][j][r] - accI[i][j][r];
                        v.y = acc3[i][j][r] - accR[i][j][r] - accI[i][j][r];
                    } else {
                        v.x = accR[i][j][r];
                        v.y = accI[i][j][r];
                    }
                    if (Pb) {
                        Pb[(int64_t)m * p.N + n] = v;
                        continue;
                    }
                    C2 *dst = Cb + p.c_moff[m] + cn;
                    if (p.accumulate) { const C2 o = *dst; v.x += o.x; v.y += o.y; }
                    *dst = v;
                }
        }
    }
}

template <typename C2>
__global__ void __launch_bounds__(256) splitk_reduce(GettArgs p) {
    const int64_t per = (int64_t)p.M * p.N;
    const int64_t total = per * p.batch;
    const C2 *P = reinterpret_cast<const C2 *>(p.part);
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
        const int b = (int)(e / per);
        const int64_t mn = e - (int64_t)b * per;
        const int m = (int)(mn / p.N), n = (int)(mn - (int64_t)m * p.N);
        if (gett_skip(p, b, m, n)) continue;  // the masked tiles wrote no partials
        double sr = 0.0, si = 0.0;
        for (int z = 0; z < p.ksplit; ++z) {
            const C2 v = P[(int64_t)z * total + e];
            sr += v.x;
            si += v.y;
        }
        C2 *dst = reinterpret_cast<C2 *>(p.C) + p.c_boff[b] + p.c_moff[m] + p.c_noff[n];
        if (p.accumulate) { sr += dst->x; si += dst->y; }
        C2 o;
        o.x = sr;
        o.y = si;
        *dst = o;
    }
}

// --------------------------------------------------------------------------
// Split-BF16: FP32 operands split into NP bf16 parts at staging time.
// MFMA 16x16x32 bf16: lane l holds A[l%16][8*(l/16) .. +8) and
// B[8*(l/16) .. +8)[l%16]; accumulator layout as the 16x16x4 forms.
__device__ inline unsigned short bf16_rne(float x) {
    unsigned int u = __float_as_uint(x);
    // round to nearest even on the upper 16 bits (inputs are finite here)
    unsigned int r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(r >> 16);
}
__device__ inline float bf16_to_f(unsigned short h) { return __uint_as_float(((unsigned int)h) << 16); }

template <int NP>
__device__ inline void split_bf16(float x, unsigned short *out) {
    float r = x;
#pragma unroll
    for (int q = 0; q < NP; ++q) {
        unsigned short h = bf16_rne(r);
        out[q] = h;
        r = r - bf16_to_f(h);
    }
}

// Split-BF16 on unpacked operands: elements gathered through the tables and
// split into bf16 parts while staging.  Used when one operand is read at most
// twice (M or N <= 128), where packing would cost more traffic than it saves.
template <int NP, int BM, int BN, int WGM, int WGN>
__global__ void __launch_bounds__(64 * WGM * WGN)
gett_bf16_direct(GettArgs p) {
    constexpr int BK = 32;
    constexpr int NT = 64 * WGM * WGN;
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int FM = WTM / 16, FN = WTN / 16;
    constexpr int LA = (BM * BK) / NT;
    constexpr int LB = (BK * BN) / NT;
    constexpr int KP = BK + 8;  // padded k extent (bf16 elements), keeps 16-byte alignment
    static_assert(LA >= 1 && LB >= 1 && NT % BK == 0 && NT >= BM && NT >= BN, "tile");
    // two LDS stages when they fit in the 160 KiB of a CU, else one
    constexpr int S = (2 * 2 * NP * (BM + BN) * KP * 2 <= 160 * 1024) ? 2 : 1;
    // planes: [stage][re/im][part][row][k]
    __shared__ __attribute__((aligned(16))) unsigned short sA[S][2][NP][BM][KP];
    __shared__ __attribute__((aligned(16))) unsigned short sB[S][2][NP][BN][KP];

    extern __shared__ int ktab[];   // non-affine k tables of the block's K slice
    const int tid = threadIdx.x;
    const int tiles_n = (p.N + BN - 1) / BN;
    const int tiles_m = (p.M + BM - 1) / BM;
    // a masked launch keeps the dispatch order, which deals consecutive tiles
    // round-robin over the XCDs: with contiguous per-XCD ranges the tiles of
    // one sample would sit on one or two XCDs and the others would idle
    const int tile = p.mask ? (int)blockIdx.x : xcd_remap(blockIdx.x, tiles_m * tiles_n);
    const int m0 = (tile / tiles_n) * BM;
    const int n0 = (tile % tiles_n) * BN;
    const int kbeg = blockIdx.z * p.kchunk;
    const int kend = min(p.K, kbeg + p.kchunk);

    int am[LA], bn[LB];
    Stager<LA> sa;
    Stager<LB> sb;
#pragma unroll
    for (int i = 0; i < LA; ++i) {
        if (p.a_kfast) { sa.kk[i] = tid % BK; am[i] = tid / BK + (NT / BK) * i; }
        else           { am[i] = tid % BM; sa.kk[i] = tid / BM + (NT / BM) * i; }
        const int m = m0 + am[i];
        sa.ro[i] = (m < p.M) ? p.a_moff[m] : -1;
    }
#pragma unroll
    for (int i = 0; i < LB; ++i) {
        if (p.b_kfast) { sb.kk[i] = tid % BK; bn[i] = tid / BK + (NT / BK) * i; }
        else           { bn[i] = tid % BN; sb.kk[i] = tid / BN + (NT / BN) * i; }
        const int n = n0 + bn[i];
        sb.ro[i] = (n < p.N) ? p.b_noff[n] : -1;
    }
    sa.ks = p.a_ks; sb.ks = p.b_ks;
    sa.kbeg = sb.kbeg = kbeg;
    sa.kend = sb.kend = kend;
    sa.kt = p.a_kaff ? nullptr : ktab;
    sb.kt = p.b_kaff ? nullptr : ktab + (p.a_kaff ? 0 : p.kchunk);
    if (!p.a_kaff) stage_ktab(ktab, p.a_koff, kbeg, kend - kbeg, tid, NT);
    if (!p.b_kaff) stage_ktab(const_cast<int *>(sb.kt), p.b_koff, kbeg, kend - kbeg, tid, NT);
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave / WGN, wn = wave % WGN;
    const float sgnA = p.conjA ? -1.f : 1.f;
    const float sgnB = p.conjB ? -1.f : 1.f;

    for (int b = blockIdx.y; b < p.batch; b += gridDim.y) {
        if (gett_skip(p, b, m0, n0)) continue;
        const __amdgpu_buffer_rsrc_t rA = make_rsrc(reinterpret_cast<const float2 *>(p.A) + p.a_boff[b], p.a_bytes);
        const __amdgpu_buffer_rsrc_t rB = make_rsrc(reinterpret_cast<const float2 *>(p.B) + p.b_boff[b], p.b_bytes);
        float2 *Cb = reinterpret_cast<float2 *>(p.C) + p.c_boff[b];
        v4f accR[FM][FN], accI[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) { accR[i][j][r] = 0.f; accI[i][j][r] = 0.f; }
        float2 ra[LA], rb[LB];
        auto gload = [&](int k0) {
            uint32_t oa[LA], ob[LB];
#pragma unroll
            for (int i = 0; i < LA; ++i) oa[i] = sa.off(i, k0, 8);
#pragma unroll
            for (int i = 0; i < LB; ++i) ob[i] = sb.off(i, k0, 8);
#pragma unroll
            for (int i = 0; i < LA; ++i) ra[i] = bload<float2>(rA, oa[i]);
#pragma unroll
            for (int i = 0; i < LB; ++i) rb[i] = bload<float2>(rB, ob[i]);
        };
        auto lstore = [&](int st) {
#pragma unroll
            for (int i = 0; i < LA; ++i) {
                unsigned short hr[NP], hi[NP];
                split_bf16<NP>(ra[i].x, hr);
                split_bf16<NP>(sgnA * ra[i].y, hi);
#pragma unroll
                for (int q = 0; q < NP; ++q) { sA[st][0][q][am[i]][sa.kk[i]] = hr[q]; sA[st][1][q][am[i]][sa.kk[i]] = hi[q]; }
            }
#pragma unroll
            for (int i = 0; i < LB; ++i) {
                unsigned short hr[NP], hi[NP];
                split_bf16<NP>(rb[i].x, hr);
                split_bf16<NP>(sgnB * rb[i].y, hi);
#pragma unroll
                for (int q = 0; q < NP; ++q) { sB[st][0][q][bn[i]][sb.kk[i]] = hr[q]; sB[st][1][q][bn[i]][sb.kk[i]] = hi[q]; }
            }
        };
        // the previous batch item's last step may still read stage 0; the first
        // pass also publishes the LDS k tables
        __syncthreads();
        gload(kbeg);
        lstore(0);
        __syncthreads();
        int st = 0;
        for (int k0 = kbeg; k0 < kend; k0 += BK) {
            const bool more = k0 + BK < kend;
            if (more) gload(k0 + BK);
            const int kc = (lane >> 4) * 8;
            v8s a[2][NP][FM], bfr[2][NP][FN];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int q = 0; q < NP; ++q) {
#pragma unroll
                    for (int i = 0; i < FM; ++i)
                        a[c][q][i] = *reinterpret_cast<const v8s *>(&sA[st][c][q][wm * WTM + i * 16 + (lane & 15)][kc]);
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        bfr[c][q][j] = *reinterpret_cast<const v8s *>(&sB[st][c][q][wn * WTN + j * 16 + (lane & 15)][kc]);
                }
            // negated imaginary parts of A for the Re C term (sign bit flip is exact)
            v8s an[NP][FM];
#pragma unroll
            for (int q = 0; q < NP; ++q)
#pragma unroll
                for (int i = 0; i < FM; ++i) an[q][i] = a[1][q][i] ^ (short)0x8000;
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
#pragma unroll
                    for (int qa = 0; qa < NP; ++qa)
#pragma unroll
                        for (int qb = 0; qb < NP; ++qb) {
                            if (qa + qb >= NP) continue;  // keep products of total order < NP
                            accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(v8bf, a[0][qa][i]), __builtin_bit_cast(v8bf, bfr[0][qb][j]), accR[i][j], 0, 0, 0);
                            accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(v8bf, an[qa][i]), __builtin_bit_cast(v8bf, bfr[1][qb][j]), accR[i][j], 0, 0, 0);
                            accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(v8bf, a[0][qa][i]), __builtin_bit_cast(v8bf, bfr[1][qb][j]), accI[i][j], 0, 0, 0);
                            accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(v8bf, a[1][qa][i]), __builtin_bit_cast(v8bf, bfr[0][qb][j]), accI[i][j], 0, 0, 0);
                        }
                }
            if (more) {
                if (S == 1) __syncthreads();  // single stage: every wave has read it
                const int nx = (S == 2) ? (st ^ 1) : 0;
                lstore(nx);
                __syncthreads();
                st = nx;
            }
        }
        float2 *Pb = p.ksplit > 1
                         ? reinterpret_cast<float2 *>(p.part) + ((int64_t)blockIdx.z * p.batch + b) * (int64_t)p.M * p.N
                         : nullptr;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int n = n0 + wn * WTN + j * 16 + (lane & 15);
            if (n >= p.N) continue;
            const int64_t cn = Pb ? 0 : p.c_noff[n];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = m0 + wm * WTM + i * 16 + (lane >> 4) * 4 + r;
                    if (m >= p.M) continue;
                    float2 v = make_float2(accR[i][j][r], accI[i][j][r]);
                    if (Pb) {
                        Pb[(int64_t)m * p.N + n] = v;
                        continue;
                    }
                    float2 *dst = Cb + p.c_moff[m] + cn;
                    if (p.accumulate) { const float2 o = *dst; v.x += o.x; v.y += o.y; }
                    *dst = v;
                }
        }
    }
}

// Packs one operand for the split-BF16 kernel: element (row, k) of batch item b
// (gathered through the plan's tables, conjugated if asked) is split into NP
// bf16 parts, stored as planes out[b][part][re/im][row][kpad], K contiguous and
// zero past K.  Done once per contraction, so the GEMM's inner loop reads ready
// bf16 fragments with 16-byte loads instead of splitting every tile it stages.
template <int NP>
__global__ void __launch_bounds__(256) k_pack_bf16(const float2 *X, const int64_t *boff, const int32_t *roff,
                                                   const int32_t *koff, int kaff, int ks, int rows, int K, int kpad,
                                                   int conj, unsigned short *out) {
    const int b = blockIdx.y;
    const int kc = kpad / 8;
    const int64_t plane = (int64_t)rows * kpad;
    const float2 *Xb = X + boff[b];
    unsigned short *Ob = out + (int64_t)b * NP * 2 * plane;
    const float sg = conj ? -1.f : 1.f;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < (int64_t)rows * kc; e += (int64_t)gridDim.x * 256) {
        const int row = (int)(e / kc), k8 = (int)(e - (int64_t)row * kc) * 8;
        const float2 *xr = Xb + roff[row];
        v8s pr[NP], pi[NP];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int k = k8 + j;
            float2 v = make_float2(0.f, 0.f);
            if (k < K) v = xr[kaff ? (int64_t)k * ks : (int64_t)koff[k]];
            unsigned short hr[NP], hi[NP];
            split_bf16<NP>(v.x, hr);
            split_bf16<NP>(sg * v.y, hi);
#pragma unroll
            for (int q = 0; q < NP; ++q) { pr[q][j] = (short)hr[q]; pi[q][j] = (short)hi[q]; }
        }
#pragma unroll
        for (int q = 0; q < NP; ++q) {
            *reinterpret_cast<v8s *>(Ob + (int64_t)(2 * q) * plane + (int64_t)row * kpad + k8) = pr[q];
            *reinterpret_cast<v8s *>(Ob + (int64_t)(2 * q + 1) * plane + (int64_t)row * kpad + k8) = pi[q];
        }
    }
}

// Split-BF16 GEMM on packed operands (see k_pack_bf16): p.A / p.B are the
// packed planes (rows M / N, p.kpad columns), p.a_bytes / p.b_bytes one batch
// item's planes.  Each stage copies 16-byte chunks (8 k values of one plane
// row) through LDS; rows past M / N read as zero (buffer range check).
template <int NP, int BM, int BN, int WGM, int WGN, bool PF2 = true>
__global__ void __launch_bounds__(64 * WGM * WGN)
gett_bf16(GettArgs p) {
    constexpr int BK = 32;
    constexpr int CH = BK / 8;  // 16-byte chunks per plane row and stage
    constexpr int NT = 64 * WGM * WGN;
    constexpr int WTM = BM / WGM, WTN = BN / WGN;
    constexpr int FM = WTM / 16, FN = WTN / 16;
    constexpr int CA = NP * 2 * BM * CH, CB = NP * 2 * BN * CH;  // chunks per stage
    constexpr int LA = (CA + NT - 1) / NT, LB = (CB + NT - 1) / NT;
    constexpr int KP = BK + 8;  // padded k extent (bf16 elements), keeps 16-byte alignment
    // two LDS stages when they fit in the 160 KiB of a CU, else one
    constexpr int S = (2 * 2 * NP * (BM + BN) * KP * 2 <= 160 * 1024) ? 2 : 1;
    // planes: [stage][re/im][part][row][k]
    __shared__ __attribute__((aligned(16))) unsigned short sA[S][2][NP][BM][KP];
    __shared__ __attribute__((aligned(16))) unsigned short sB[S][2][NP][BN][KP];

    const int tid = threadIdx.x;
    const int tiles_n = (p.N + BN - 1) / BN;
    const int tiles_m = (p.M + BM - 1) / BM;
    // a masked launch keeps the dispatch order, which deals consecutive tiles
    // round-robin over the XCDs: with contiguous per-XCD ranges the tiles of
    // one sample would sit on one or two XCDs and the others would idle
    const int tile = p.mask ? (int)blockIdx.x : xcd_remap(blockIdx.x, tiles_m * tiles_n);
    const int m0 = (tile / tiles_n) * BM;
    const int n0 = (tile % tiles_n) * BN;
    const int kbeg = blockIdx.z * p.kchunk;
    const int kend = min(p.K, kbeg + p.kchunk);
    const int64_t planeA = (int64_t)p.M * p.kpad, planeB = (int64_t)p.N * p.kpad;

    // chunk e = (plane q*2+c, row in a tile of tr rows, ch) -> byte offset in one
    // batch item's planes, or OOB past the matrix
    auto chunk_off = [&](int e, int tr, int rows, int r0, int64_t plane, int k0) {
        const int ch = e % CH, row = (e / CH) % tr, pl = e / (CH * tr);
        if (r0 + row >= rows) return OOB;
        return (uint32_t)(((int64_t)pl * plane + (int64_t)(r0 + row) * p.kpad + k0 + ch * 8) * 2);
    };
    const int wave = tid >> 6, lane = tid & 63;
    const int wm = wave / WGN, wn = wave % WGN;

    for (int b = blockIdx.y; b < p.batch; b += gridDim.y) {
        if (gett_skip(p, b, m0, n0)) continue;
        const __amdgpu_buffer_rsrc_t rA =
            make_rsrc(reinterpret_cast<const unsigned short *>(p.A) + (int64_t)b * NP * 2 * planeA, p.a_bytes);
        const __amdgpu_buffer_rsrc_t rB =
            make_rsrc(reinterpret_cast<const unsigned short *>(p.B) + (int64_t)b * NP * 2 * planeB, p.b_bytes);
        float2 *Cb = reinterpret_cast<float2 *>(p.C) + p.c_boff[b];
        v4f accR[FM][FN], accI[FM][FN];
#pragma unroll
        for (int i = 0; i < FM; ++i)
#pragma unroll
            for (int j = 0; j < FN; ++j)
#pragma unroll
                for (int r = 0; r < 4; ++r) { accR[i][j][r] = 0.f; accI[i][j][r] = 0.f; }
        // operand chunks are prefetched two k-steps ahead into alternating
        // register sets (PF2): one k-step of MFMA work is shorter than a global
        // load's latency, so a single step of lead leaves the CU waiting at the
        // barrier; tiles short of registers keep one set and one step of lead
        v8s ra0[LA], rb0[LB], ra1[PF2 ? LA : 1], rb1[PF2 ? LB : 1];
        // loads are issued on every step (past kend they read the zero of an
        // out-of-range offset): a branch around them would leave the count of
        // loads in flight unknown at the LDS store, and the wait there would
        // then also cover the loads just issued for the step after next
        auto gload = [&](int k0, v8s (&ra)[LA], v8s (&rb)[LB]) {
            const bool in = k0 < kend;
#pragma unroll
            for (int i = 0; i < LA; ++i) {
                const int e = tid + NT * i;
                const uint32_t o = (in && e < CA) ? chunk_off(e, BM, p.M, m0, planeA, k0) : OOB;
                ra[i] = __builtin_bit_cast(v8s, __builtin_amdgcn_raw_buffer_load_b128(rA, (int)o, 0, 0));
            }
#pragma unroll
            for (int i = 0; i < LB; ++i) {
                const int e = tid + NT * i;
                const uint32_t o = (in && e < CB) ? chunk_off(e, BN, p.N, n0, planeB, k0) : OOB;
                rb[i] = __builtin_bit_cast(v8s, __builtin_amdgcn_raw_buffer_load_b128(rB, (int)o, 0, 0));
            }
        };
        auto lstore = [&](int st, const v8s (&ra)[LA], const v8s (&rb)[LB]) {
#pragma unroll
            for (int i = 0; i < LA; ++i) {
                const int e = tid + NT * i;
                if (e >= CA) continue;
                const int ch = e % CH, row = (e / CH) % BM, pl = e / (CH * BM);
                *reinterpret_cast<v8s *>(&sA[st][pl & 1][pl >> 1][row][ch * 8]) = ra[i];
            }
#pragma unroll
            for (int i = 0; i < LB; ++i) {
                const int e = tid + NT * i;
                if (e >= CB) continue;
                const int ch = e % CH, row = (e / CH) % BN, pl = e / (CH * BN);
                *reinterpret_cast<v8s *>(&sB[st][pl & 1][pl >> 1][row][ch * 8]) = rb[i];
            }
        };
        auto compute = [&](int st) {
            const int kc = (lane >> 4) * 8;
            v8s a[2][NP][FM], bfr[2][NP][FN];
#pragma unroll
            for (int c = 0; c < 2; ++c)
#pragma unroll
                for (int q = 0; q < NP; ++q) {
#pragma unroll
                    for (int i = 0; i < FM; ++i)
                        a[c][q][i] = *reinterpret_cast<const v8s *>(&sA[st][c][q][wm * WTM + i * 16 + (lane & 15)][kc]);
#pragma unroll
                    for (int j = 0; j < FN; ++j)
                        bfr[c][q][j] = *reinterpret_cast<const v8s *>(&sB[st][c][q][wn * WTN + j * 16 + (lane & 15)][kc]);
                }
            // negated imaginary parts of A for the Re C term (sign bit flip is exact)
            v8s an[NP][FM];
#pragma unroll
            for (int q = 0; q < NP; ++q)
#pragma unroll
                for (int i = 0; i < FM; ++i)
                    an[q][i] = __builtin_bit_cast(v8s, __builtin_bit_cast(v4u, a[1][q][i]) ^ 0x80008000u);
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int j = 0; j < FN; ++j) {
#pragma unroll
                    for (int qa = 0; qa < NP; ++qa)
#pragma unroll
                        for (int qb = 0; qb < NP; ++qb) {
                            if (qa + qb >= NP) continue;  // keep products of total order < NP
                            accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(v8bf, a[0][qa][i]), __builtin_bit_cast(v8bf, bfr[0][qb][j]), accR[i][j], 0, 0, 0);
                            accR[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(v8bf, an[qa][i]), __builtin_bit_cast(v8bf, bfr[1][qb][j]), accR[i][j], 0, 0, 0);
                            accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(v8bf, a[0][qa][i]), __builtin_bit_cast(v8bf, bfr[1][qb][j]), accI[i][j], 0, 0, 0);
                            accI[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(
                                __builtin_bit_cast(v8bf, a[1][qa][i]), __builtin_bit_cast(v8bf, bfr[0][qb][j]), accI[i][j], 0, 0, 0);
                        }
                }
        };
        int st = 0;
        // one k-step: `cur` holds step k0 + BK (loaded a step earlier), `nxt`
        // receives step k0 + 2 BK
        auto step = [&](int k0, v8s (&cur_a)[LA], v8s (&cur_b)[LB], v8s (&nxt_a)[LA], v8s (&nxt_b)[LB]) {
            gload(k0 + 2 * BK, nxt_a, nxt_b);
            if (k0 < kend) compute(st);
            if (k0 + BK < kend) {
                if (S == 1) __syncthreads();  // single stage: every wave has read it
                const int nx = (S == 2) ? (st ^ 1) : 0;
                lstore(nx, cur_a, cur_b);
                __syncthreads();
                st = nx;
            }
        };
        // the previous batch item's last step may still read stage 0
        __syncthreads();
        gload(kbeg, ra0, rb0);
        lstore(0, ra0, rb0);
        if constexpr (PF2) {
            gload(kbeg + BK, ra0, rb0);
            __syncthreads();
            // both halves run on every trip (the second is idle past kend) so
            // that every trip issues the same loads
            for (int k0 = kbeg; k0 < kend; k0 += 2 * BK) {
                step(k0, ra0, rb0, ra1, rb1);
                step(k0 + BK, ra1, rb1, ra0, rb0);
            }
        } else {
            __syncthreads();
            for (int k0 = kbeg; k0 < kend; k0 += BK) {
                const bool more = k0 + BK < kend;
                if (more) gload(k0 + BK, ra0, rb0);
                compute(st);
                if (more) {
                    if (S == 1) __syncthreads();
                    const int nx = (S == 2) ? (st ^ 1) : 0;
                    lstore(nx, ra0, rb0);
                    __syncthreads();
                    st = nx;
                }
            }
        }
        float2 *Pb = p.ksplit > 1
                         ? reinterpret_cast<float2 *>(p.part) + ((int64_t)blockIdx.z * p.batch + b) * (int64_t)p.M * p.N
                         : nullptr;
#pragma unroll
        for (int j = 0; j < FN; ++j) {
            const int n = n0 + wn * WTN + j * 16 + (lane & 15);
            if (n >= p.N) continue;
            const int64_t cn = Pb ? 0 : p.c_noff[n];
#pragma unroll
            for (int i = 0; i < FM; ++i)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int m = m0 + wm * WTM + i * 16 + (lane >> 4) * 4 + r;
                    if (m >= p.M) continue;
                    float2 v = make_float2(accR[i][j][r], accI[i][j][r]);
                    if (Pb) {
                        Pb[(int64_t)m * p.N + n] = v;
                        continue;
                    }
                    float2 *dst = Cb + p.c_moff[m] + cn;
                    if (p.accumulate) { const float2 o = *dst; v.x += o.x; v.y += o.y; }
                    *dst = v;
                }
        }
    }
}

template <typename K>
hipError_t launch_k(K kernel, const GettArgs &a, int bm, int bn, int nt, hipStream_t s) {
    const int tiles = ((a.M + bm - 1) / bm) * ((a.N + bn - 1) / bn);
    const int gy = a.batch < 65535 ? a.batch : 65535;
    if (tiles <= 0 || a.batch <= 0) return hipSuccess;
    const int gz = a.ksplit > 1 ? a.ksplit : 1;
    if ((!a.a_kaff || !a.b_kaff) && a.kchunk > GETT_KTAB) return hipErrorInvalidValue;
    if (a.mask && ((a.mask_mode == 2 && a.mask_div % bm) || (a.mask_mode == 3 && a.mask_div % bn)))
        return hipErrorInvalidValue;  // launch_gett clears a mask the tiles do not align with
    const size_t dyn = (size_t)((a.a_kaff ? 0 : a.kchunk) + (a.b_kaff ? 0 : a.kchunk)) * sizeof(int);
    static bool attr = false;  // one per kernel instantiation
    if (!attr) {
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(kernel),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize,
                                                 (int)(2 * GETT_KTAB * sizeof(int)));
        if (e != hipSuccess) return e;
        attr = true;
    }
    hipLaunchKernelGGL(kernel, dim3(tiles, gy, gz), dim3(nt), dyn, s, a);
    return hipGetLastError();
}

template <typename C2>
hipError_t launch_reduce(const GettArgs &a, hipStream_t s) {
    if (a.ksplit <= 1) return hipSuccess;
    const int64_t total = (int64_t)a.M * a.N * a.batch;
    int64_t g = (total + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(splitk_reduce<C2>, dim3((unsigned)g), dim3(256), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_pack_bf16(int np, const void *X, const int64_t *boff, const int32_t *roff, const int32_t *koff,
                            int kaff, int ks, int rows, int K, int kpad, int batch, int conj, void *out,
                            hipStream_t s) {
    if (rows <= 0 || batch <= 0) return hipSuccess;
    const int64_t work = (int64_t)rows * (kpad / 8);
    int64_t g = (work + 255) / 256;
    if (g > 8192) g = 8192;
    const int gy = batch < 65535 ? batch : 65535;
    if (batch > gy) return hipErrorInvalidValue;
    auto x = reinterpret_cast<const float2 *>(X);
    auto o = reinterpret_cast<unsigned short *>(out);
    if (np == 2)
        hipLaunchKernelGGL(k_pack_bf16<2>, dim3((unsigned)g, gy), dim3(256), 0, s, x, boff, roff, koff, kaff, ks, rows,
                           K, kpad, conj, o);
    else
        hipLaunchKernelGGL(k_pack_bf16<3>, dim3((unsigned)g, gy), dim3(256), 0, s, x, boff, roff, koff, kaff, ks, rows,
                           K, kpad, conj, o);
    return hipGetLastError();
}

void gett_tile(int cfg, int prec, int *bm, int *bn) {
    switch (cfg) {
        case CFG_64x64: *bm = 64; *bn = 64; break;
        case CFG_128x64: *bm = 128; *bn = 64; break;
        case CFG_64x16: *bm = 64; *bn = 16; break;
        case CFG_128x64W: *bm = 128; *bn = 64; break;
        case CFG_128x128W: *bm = 128; *bn = 128; break;
        default: *bm = 64; *bn = 64; break;
    }
    (void)prec;
}

static hipError_t launch_main(const GettArgs &a, int prec, int cfg, hipStream_t s);

hipError_t launch_gett(const GettArgs &a0, int prec, int cfg, hipStream_t s) {
    if (a0.M <= 0 || a0.N <= 0 || a0.batch <= 0) return hipSuccess;
    GettArgs a = a0;
    if (a.mask) {
        // tiles that would straddle mask items: compute everything
        int bm = 64, bn = 64;
        gett_tile(cfg, prec, &bm, &bn);
        if (a.mask_div <= 0 || a.mask_mode < 1 || a.mask_mode > 3 || (a.mask_mode == 2 && a.mask_div % bm) ||
            (a.mask_mode == 3 && a.mask_div % bn))
            a.mask = nullptr;
    }
    hipError_t e = launch_main(a, prec, cfg, s);
    if (e != hipSuccess || a.ksplit <= 1) return e;
    return prec == P_FP64 ? launch_reduce<double2>(a, s) : launch_reduce<float2>(a, s);
}

static hipError_t launch_main(const GettArgs &a, int prec, int cfg, hipStream_t s) {
    if (prec == P_FP64) {
        switch (cfg) {
            case CFG_64x64: return launch_k(gett_mfma<double, 64, 64, 16, 2, 2, GAUSS3M>, a, 64, 64, 256, s);
            case CFG_128x64: return launch_k(gett_mfma<double, 128, 64, 16, 2, 2, false>, a, 128, 64, 256, s);
            case CFG_64x16: return launch_k(gett_mfma<double, 64, 16, 16, 4, 1, GAUSS3M>, a, 64, 16, 256, s);
            case CFG_128x64W: return launch_k(gett_mfma<double, 128, 64, 16, 4, 2, GAUSS3M>, a, 128, 64, 512, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (prec == P_FP32) {
        switch (cfg) {
            case CFG_64x64: return launch_k(gett_mfma<float, 64, 64, 16, 2, 2, GAUSS3M>, a, 64, 64, 256, s);
            case CFG_128x64: return launch_k(gett_mfma<float, 128, 64, 16, 2, 2, false>, a, 128, 64, 256, s);
            case CFG_64x16: return launch_k(gett_mfma<float, 64, 16, 16, 4, 1, GAUSS3M>, a, 64, 16, 256, s);
            case CFG_128x64W: return launch_k(gett_mfma<float, 128, 64, 16, 4, 2, GAUSS3M>, a, 128, 64, 512, s);
            default: return hipErrorInvalidValue;
        }
    }
    if (prec == P_BF16X3) {
        switch (cfg) {
            case CFG_64x64: return a.kpad ? launch_k(gett_bf16<2, 64, 64, 2, 2>, a, 64, 64, 256, s)
                                          : launch_k(gett_bf16_direct<2, 64, 64, 2, 2>, a, 64, 64, 256, s);
            case CFG_128x64: return a.kpad ? launch_k(gett_bf16<2, 128, 64, 2, 2>, a, 128, 64, 256, s)
                                           : launch_k(gett_bf16_direct<2, 128, 64, 2, 2>, a, 128, 64, 256, s);
            case CFG_64x16: return a.kpad ? launch_k(gett_bf16<2, 64, 16, 4, 1>, a, 64, 16, 256, s)
                                          : launch_k(gett_bf16_direct<2, 64, 16, 4, 1>, a, 64, 16, 256, s);
            case CFG_128x64W: return a.kpad ? launch_k(gett_bf16<2, 128, 64, 4, 2>, a, 128, 64, 512, s)
                                            : launch_k(gett_bf16_direct<2, 128, 64, 4, 2>, a, 128, 64, 512, s);
            case CFG_128x128W: return a.kpad ? launch_k(gett_bf16<2, 128, 128, 2, 4, false>, a, 128, 128, 512, s)
                                             : hipErrorInvalidValue;
            default: return hipErrorInvalidValue;
        }
    }
    switch (cfg) {
        case CFG_64x64: return a.kpad ? launch_k(gett_bf16<3, 64, 64, 2, 2>, a, 64, 64, 256, s)
                                      : launch_k(gett_bf16_direct<3, 64, 64, 2, 2>, a, 64, 64, 256, s);
        case CFG_128x64: return a.kpad ? launch_k(gett_bf16<3, 128, 64, 2, 2>, a, 128, 64, 256, s)
                                       : launch_k(gett_bf16_direct<3, 128, 64, 2, 2>, a, 128, 64, 256, s);
        case CFG_64x16: return a.kpad ? launch_k(gett_bf16<3, 64, 16, 4, 1>, a, 64, 16, 256, s)
                                      : launch_k(gett_bf16_direct<3, 64, 16, 4, 1>, a, 64, 16, 256, s);
        case CFG_128x64W: return a.kpad ? launch_k(gett_bf16<3, 128, 64, 4, 2>, a, 128, 64, 512, s)
                                        : launch_k(gett_bf16_direct<3, 128, 64, 4, 2>, a, 128, 64, 512, s);
        case CFG_128x128W: return a.kpad ? launch_k(gett_bf16<3, 128, 128, 2, 4, false>, a, 128, 128, 512, s)
                                         : hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
    }
}

}  // namespace tnk
