// Sequential bitstring sampling from the stored norm boundaries (Appendix,
// "Sampling from a Tensor Network State", Fig. 7d).
//
// Samples run in waves of Z in flight; every per-sample tensor carries a
// leading sample index z.  For a row b:
//  * right environments [z, a, b, g, h, k] of (amplitude boundary m, its
//    conjugate, the row's ket and bra tensors, the stored norm boundary below)
//    are built right to left;
//  * qubit by qubit, the left environment is extended with the site projected
//    on s = 0 and s = 1 in ket and bra (the bra/ket bond of the open site split),
//    closed against the right environment to give P~(s), the bit is drawn, and
//    the environment projected on the drawn bit is kept;
//  * the product of m with the projected row x_b . psi_b is fitted to a new m of
//    bond <= chi_x by the one-site fit (single layer);
//  * optionally (svd_cutoff > 0) the fitted m is truncated per sample by a
//    left-to-right SVD sweep that keeps the fewest singular values whose
//    discarded weight is within the cutoff (clamped to [chi_x_min, width]);
//    the dropped directions stay as zeros, so every sample of a wave keeps the
//    same tensor shapes while its effective bond varies.
// q(x) accumulates the drawn conditionals; p(x) is the last amplitude boundary
// contracted with the last projected row.  Probabilities are FP64; P(s) =
// max(Re P~(s), 0) / sum, x = 0 iff u < P(0).
#include <algorithm>
#include <cstdio>
#include <cmath>
#include <vector>

#include "tn_core.hpp"

namespace tnb {

namespace {

constexpr int ENV_RENORM = 4;  // sites between rescalings of the sampler's environments

// First contraction of a left step, shared by both projections: L . m.
// Direct route: [z,b,g,h,k,u,A]; transfer-matrix route (u = 1): [z,A,b,g,h,k].
Ten left_t1(Engine &E, const Ten &L, const Ten &m, bool via_T) {
    return E.contract_new(op(L, "zabghk"), op(m, "zauA"), via_T ? "zAbghk" : "zbghkuA");
}

// Rest of a left step with the site projected on s, from t1 (direct route).
Ten left_rest(Engine &E, const Ten &t1, const Ten &m, const SiteRef &a, const Ten &B, int s) {
    Ten t2 = E.contract_new(op(t1, "zbghkuA"), sop_proj(a, s, "uhdH"), "zbgkAdH");
    Ten t3 = E.contract_new(op(t2, "zbgkAdH"), op(B, "gdeG"), "zbkAHeG");
    E.drop(t2);
    Ten W = E.contract_new(op(m, "zbvB", true), sop_proj(a, s, "vkeK", true), "zbBkeK");
    Ten out = E.contract_new(op(t3, "zbkAHeG"), op(W, "zbBkeK"), "zABGHK");
    E.drop(t3);
    E.drop(W);
    return out;
}

// Rest of a left step through a u = 1 site with transfer matrix T_s, from t1.
Ten left_rest_T(Engine &E, const Ten &t1, const Ten &m, const Ten &T) {
    Ten t2 = E.contract_new(op(t1, "zAbghk"), op(T, "ghkGHK"), "zAbGHK");
    Ten out = E.contract_new(op(t2, "zAbGHK"), op(m, "zbvB", true), "zABGHK");
    E.drop(t2);
    return out;
}

// Left step with the physical index summed (sites without a qubit):
// [z,a,b,g,h,k] + column -> [z,A,B,G,H,K].
Ten env_left_traced(Engine &E, const Ten &L, const Ten &m, const SiteRef &a, const Ten &B) {
    Ten t1 = left_t1(E, L, m, false);
    Ten t2 = E.contract_new(op(t1, "zbghkuA"), sop(a, "suhdH"), "zbgkAsdH");
    E.drop(t1);
    Ten t3 = E.contract_new(op(t2, "zbgkAsdH"), op(B, "gdeG"), "zbkAsHeG");
    E.drop(t2);
    Ten W = E.contract_new(op(m, "zbvB", true), sop(a, "svkeK", true), "zbBskeK");
    Ten out = E.contract_new(op(t3, "zbkAsHeG"), op(W, "zbBskeK"), "zABGHK");
    E.drop(t3);
    E.drop(W);
    return out;
}

// [z,A,B,G,H,K] + column -> [z,a,b,g,h,k] (physical index summed).
Ten env_right(Engine &E, const Ten &R, const Ten &m, const SiteRef &a, const Ten &B) {
    Ten t1 = E.contract_new(op(m, "zauA"), op(R, "zABGHK"), "zauBGHK");
    Ten t2 = E.contract_new(op(t1, "zauBGHK"), sop(a, "suhdH"), "zaBGKshd");
    E.drop(t1);
    Ten t3 = E.contract_new(op(t2, "zaBGKshd"), op(B, "gdeG"), "zaBKshge");
    E.drop(t2);
    Ten W = E.contract_new(op(m, "zbvB", true), sop(a, "svkeK", true), "zbBskeK");
    Ten out = E.contract_new(op(t3, "zaBKshge"), op(W, "zbBskeK"), "zabghk");
    E.drop(t3);
    E.drop(W);
    return out;
}

// Sites without an up bond (u = 1) let the ket and bra row tensors and the norm
// boundary below be contracted into a sample-independent column transfer
// matrix T_s[g,h,k,G,H,K] = sum_{d,e} B[g,d,e,G] A[s,h,d,H] conj(A[s,k,e,K])
// (s < 0: summed over s).  An environment step is then one square GEMM over
// (g,h,k) shared by every sample of the wave, instead of contracting B, A and
// conj(A) per sample.
Ten transfer(Engine &E, const SiteRef &a, const Ten &B, int s) {
    if (s < 0) {
        Ten x1 = E.contract_new(op(B, "gdeG"), sop(a, "suhdH"), "geGshH");
        Ten T = E.contract_new(op(x1, "geGshH"), sop(a, "sukeK", true), "ghkGHK");
        E.drop(x1);
        return T;
    }
    Ten x1 = E.contract_new(op(B, "gdeG"), sop_proj(a, s, "uhdH"), "geGhH");
    Ten T = E.contract_new(op(x1, "geGhH"), sop_proj(a, s, "ukeK", true), "ghkGHK");
    E.drop(x1);
    return T;
}

// Left step through a u = 1 site with its transfer matrix: [z,a,b,g,h,k] -> [z,A,B,G,H,K].
Ten env_left_T(Engine &E, const Ten &L, const Ten &m, const Ten &T) {
    Ten t1 = left_t1(E, L, m, true);
    Ten out = left_rest_T(E, t1, m, T);
    E.drop(t1);
    return out;
}

// Right step through a u = 1 site: [z,A,B,G,H,K] -> [z,a,b,g,h,k].
Ten env_right_T(Engine &E, const Ten &R, const Ten &m, const Ten &T) {
    Ten t1 = E.contract_new(op(R, "zABGHK"), op(m, "zbvB", true), "zAbGHK");
    Ten t2 = E.contract_new(op(t1, "zAbGHK"), op(T, "ghkGHK"), "zAbghk");
    E.drop(t1);
    Ten out = E.contract_new(op(m, "zauA"), op(t2, "zAbghk"), "zabghk");
    E.drop(t2);
    return out;
}

// Cost model (multiply-adds per sample for one left step with both projections)
// of the direct order against the transfer-matrix route, which needs u = 1 and
// a transfer matrix of modest size.
bool transfer_pays(const SiteRef &a, const Ten &B, const Ten &m) {
    if (a.dim(1) != 1) return false;
    const double x = std::max(m.d[1], m.d[3]);
    const double g = B.d[0], G = B.d[3], h = a.dim(2), H = a.dim(4), d = a.dim(3), p = a.dim(0);
    const double tsize = g * h * h * G * H * H;
    if (tsize > (double)(1 << 26)) return false;
    const double direct = x * x * x * g * h * h + x * x * g * h * p * d * H * h + x * x * h * p * H * d * G * g * d +
                          x * x * x * G * H * H * h * p * d;
    const double viaT = x * x * x * g * h * h + p * x * x * g * h * h * G * H * H + p * x * x * x * G * H * H;
    return viaT < direct;
}

void unit(Engine &E, Ten &t, int Z, double *logacc = nullptr) {
    const int64_t per = t.numel() / Z;
    E.normalise(t.p, t.esz, per, Z, per, logacc, logacc != nullptr, nullptr);
}

// Single-layer one-site fit of m . X (batched over z) to bond <= chi_x.
// m[c]: [z, a, u, A]; X[c]: [z, u, h, d, H]; returns [z, y, d, Y]; mlog += log ||.||.
std::vector<Ten> fit_single(Engine &E, const std::vector<Ten> &m, const std::vector<Ten> &X, const SampleOpts &o,
                            int row, const uint64_t *sample_idx, double *mlog) {
    const int L = (int)X.size();
    const int Z = X[0].d[0];
    std::vector<int> phys(L);
    std::vector<int64_t> bin(std::max(L - 1, 0));
    for (int c = 0; c < L; ++c) phys[c] = X[c].d[3];
    for (int c = 0; c + 1 < L; ++c) bin[c] = (int64_t)m[c].d[3] * X[c].d[4];
    bool exact;
    std::vector<int> t;
    plan_bonds(phys, bin, o.chi_x, exact, t);
    std::vector<Ten> Y(L);
    if (exact && !o.force_fit) {
        for (int c = 0; c < L; ++c) {
            Ten e = E.contract_new(op(m[c], "zauA"), op(X[c], "zuhdH"), "zahdAH");
            e.d = {Z, m[c].d[1] * X[c].d[2], X[c].d[3], m[c].d[3] * X[c].d[4]};
            Y[c] = e;
        }
        canonicalise(E, Y, 1, mlog, true);
        return Y;
    }
    for (int c = 0; c < L; ++c) {
        const int tl = c > 0 ? t[c - 1] : 1, tr = c + 1 < L ? t[c] : 1;
        Y[c] = E.make({Z, tl, phys[c], tr});
        const int64_t per = Y[c].numel() / Z;
        TN_HIP(tnk::launch_init_tensor(Y[c].p, Y[c].esz, per, Z, per, o.init_seed, (uint64_t)o.init_tag,
                                       (uint64_t)row, (uint64_t)c, sample_idx, E.s));
    }
    right_canonicalise(E, Y, 1);
    auto rpart = [&](const Ten &R, int c) {  // [z,a,h,d,Y]
        Ten t1 = E.contract_new(op(m[c], "zauA"), op(R, "zYAH"), "zauYH");
        Ten tr = E.contract_new(op(t1, "zauYH"), op(X[c], "zuhdH"), "zahdY");
        E.drop(t1);
        return tr;
    };
    auto lpart = [&](const Ten &Lf, int c) {  // [z,y,A,d,H]
        Ten t1 = E.contract_new(op(Lf, "zyah"), op(m[c], "zauA"), "zyhuA");
        Ten tl = E.contract_new(op(t1, "zyhuA"), op(X[c], "zuhdH"), "zyAdH");
        E.drop(t1);
        return tl;
    };
    std::vector<Ten> Le(L + 1), Re(L + 1);
    Re[L] = ones(E, {Z, 1, 1, 1});
    Le[0] = ones(E, {Z, 1, 1, 1});
    for (int c = L - 1; c >= 1; --c) {
        Ten tr = rpart(Re[c + 1], c);
        Re[c] = E.contract_new(op(Y[c], "zydY", true), op(tr, "zahdY"), "zyah");
        E.drop(tr);
    }
    for (int sw = 0; sw < o.sweeps; ++sw) {
        for (int c = 0; c + 1 < L; ++c) {
            Ten tl = lpart(Le[c], c);
            Ten N = E.contract_new(op(tl, "zyAdH"), op(Re[c + 1], "zYAH"), "zydY");
            Ten Q;
            qr_left(E, N, 1, Q, nullptr);
            E.drop(N);
            E.drop(Y[c]);
            Y[c] = Q;
            if (Le[c + 1].p) E.drop(Le[c + 1]);
            Le[c + 1] = E.contract_new(op(Y[c], "zydY", true), op(tl, "zyAdH"), "zYAH");
            E.drop(tl);
        }
        for (int c = L - 1; c >= 1; --c) {
            Ten tr = rpart(Re[c + 1], c);
            Ten N = E.contract_new(op(Le[c], "zyah"), op(tr, "zahdY"), "zydY");
            Ten Q;
            lq_right(E, N, 1, Q, nullptr);
            E.drop(N);
            E.drop(Y[c]);
            Y[c] = Q;
            if (Re[c].p) E.drop(Re[c]);
            Re[c] = E.contract_new(op(Y[c], "zydY", true), op(tr, "zahdY"), "zyah");
            E.drop(tr);
        }
    }
    {
        Ten tr = rpart(Re[1], 0);
        Ten N = E.contract_new(op(Le[0], "zyah"), op(tr, "zahdY"), "zydY");
        E.drop(tr);
        E.drop(Y[0]);
        Y[0] = N;
    }
    for (auto &x : Le)
        if (x.p) E.drop(x);
    for (auto &x : Re)
        if (x.p) E.drop(x);
    unit(E, Y[0], Z, mlog);
    return Y;
}

// Left-to-right SVD truncation of the fitted amplitude boundary m (sites 1..L-1
// right-canonical, the gauge the fit and the exact product leave).  At cut c:
// Householder QR of site c as (a u) x A (FP64, rank-deficient input allowed),
// Jacobi SVD of R with the keep rule, site c <- Q U_k and site c+1 <- S_k V_k^H
// site c+1, zero past k.  kbuf [cuts][Z] receives the kept counts.
void truncate_cutoff(Engine &E, std::vector<Ten> &m, const SampleOpts &o, int *kbuf) {
    const int L = (int)m.size();
    const int Z = m[0].d[0];
    for (int c = 0; c + 1 < L; ++c) {
        const int a = m[c].d[1], u = m[c].d[2], A = m[c].d[3];
        const int64_t rows = (int64_t)a * u;
        if (A > tnk::SVD_NMAX)
            throw TnError(ST_UNSUPPORTED, "SVD truncation supports bonds up to " + std::to_string(tnk::SVD_NMAX));
        if (rows < A) throw TnError(ST_SHAPE, "amplitude boundary site narrower than its right bond");
        Ten Q = E.make({Z, a, u, A});
        Ten R = E.make({Z, A, A}, 16);
        tnk::QrArgs q{};
        q.m = (int)rows; q.n = A; q.batch = Z;
        q.A = m[c].p; q.a_esz = m[c].esz; q.a_bs = rows * A; q.a_rs = A; q.a_cs = 1; q.a_conj = 0;
        q.Q = Q.p; q.q_esz = Q.esz; q.q_bs = rows * A; q.q_rs = A; q.q_cs = 1; q.q_conj = 0;
        q.R = R.p; q.r_esz = 16; q.r_bs = (int64_t)A * A; q.r_rs = A; q.r_cs = 1; q.r_conj = 0;
        E.qr(q);
        Ten U = E.make({Z, A, A}), SV = E.make({Z, A, A});
        const size_t wsb = tnk::svd_trunc_workspace_bytes(A, Z);
        void *ws = wsb ? E.raw(wsb) : nullptr;
        const hipError_t err = tnk::launch_svd_trunc(static_cast<const double *>(R.p), A, Z, o.svd_cutoff, o.chi_x_min,
                                                     U.p, SV.p, U.esz, kbuf + (size_t)c * Z, ws, E.s);
        if (ws) E.unraw(ws);
        TN_HIP(err);
        E.drop(R);
        Ten mc = E.contract_new(op(Q, "zauk"), op(U, "zkA"), "zauA");
        E.drop(Q);
        E.drop(U);
        Ten mn = E.contract_new(op(SV, "zAk"), op(m[c + 1], "zkvB"), "zAvB");
        E.drop(SV);
        E.drop(m[c]);
        E.drop(m[c + 1]);
        m[c] = mc;
        m[c + 1] = mn;
    }
}

// <x|psi> from the last amplitude boundary and the last projected row (whose
// down legs have dimension 1): log_p[z] = 2 (mlog[z] + log|v_z|), arg[z] =
// arg v_z (optional); amp is [Z] complex128 scratch.
void last_row_amplitude(Engine &E, const std::vector<Ten> &m, const std::vector<Ten> &X, double *mlog, double *amp,
                        double *log_p, double *arg) {
    const int cols = (int)X.size();
    const int Z = X[0].d[0];
    Ten v = ones(E, {Z, 1, 1});
    for (int c = 0; c < cols; ++c) {
        Ten t1 = E.contract_new(op(v, "zah"), op(m[c], "zauA"), "zhuA");
        Ten Xc = X[c];
        Xc.d = {Z, X[c].d[1], X[c].d[2], X[c].d[4]};
        Ten v2 = E.contract_new(op(t1, "zhuA"), op(Xc, "zuhH"), "zAH");
        E.drop(t1);
        E.drop(v);
        v = v2;
        if (c + 1 < cols) unit(E, v, Z, mlog);
    }
    TN_HIP(tnk::launch_convert(v.p, v.esz, amp, 16, Z, E.s));
    TN_HIP(tnk::launch_logp(amp, mlog, Z, log_p, arg, E.s));
    E.drop(v);
}

// Peak bytes per sample in flight for row sampling (right envs + intermediates).
double bytes_per_sample(const LView &V, const BoundarySet &B, int chi_x, int esz) {
    double peak = 0;
    for (int r = 0; r < V.rows; ++r) {
        double envs = 0, inter = 0;
        for (int c = 0; c < V.cols; ++c) {
            const SiteRef &a = V.at(r, c);
            const double x = std::min<double>(chi_x, 1 << 20);
            const double g = B.below[r].site[c].d[0], G = B.below[r].site[c].d[3];
            const double u = a.dim(1), h = a.dim(2), d = a.dim(3), H = a.dim(4), p = a.dim(0);
            envs += x * x * G * H * H;
            const double t2 = x * x * G * H * p * h * d;   // right env S2
            const double t3 = x * x * H * p * h * g * d;   // right env S3
            const double w = x * x * p * h * d * H * u;
            inter = std::max(inter, t2 + t3 + w + x * x * g * h * h * 3);
        }
        peak = std::max(peak, envs + inter);
    }
    return peak * esz * 1.3;
}

}  // namespace

void sample(Engine &E, const PepsDev &P, const BoundarySet &B, const SampleOpts &o, uint64_t first, int64_t n,
            const double *uniforms, uint8_t *bits, double *log_q, double *log_p, int *chi_used) {
    const LView V = make_view(P, 0);
    const int rows = V.rows, cols = V.cols;
    int Zw = o.wave;
    if (Zw <= 0) {
        size_t freeb = 0, total = 0;
        TN_HIP(hipMemGetInfo(&freeb, &total));
        const double per = bytes_per_sample(V, B, o.chi_x, E.esz);
        const double budget = 0.5 * (double)freeb + 0.5 * (double)E.held();
        Zw = (int)std::max(1.0, std::min(4096.0, std::floor(budget / std::max(per, 1.0))));
    }
    Zw = (int)std::min<int64_t>(Zw, n);
    // per-wave device state
    uint64_t *sidx = reinterpret_cast<uint64_t *>(E.raw((size_t)Zw * 8));
    double *mlog = reinterpret_cast<double *>(E.raw((size_t)Zw * 8));
    double *pt = reinterpret_cast<double *>(E.raw((size_t)Zw * 32));
    double *ptot = reinterpret_cast<double *>(E.raw((size_t)Zw * 16));
    double *ptd = reinterpret_cast<double *>(E.raw((size_t)Zw * 16));
    int *need = reinterpret_cast<int *>(E.raw((size_t)Zw * 4));
    // below this fraction of the traced total, the other bit's P~ taken as a
    // difference is not trusted: a few hundred unit roundoffs of the GEMM mode
    const double diff_thr = E.prec == tnk::P_FP64 ? 1e-12 : (E.prec == tnk::P_BF16X3 ? 1e-2 : 1e-4);
    double *lnR = reinterpret_cast<double *>(E.raw((size_t)Zw * 8 * (cols + 1)));
    int *flags = reinterpret_cast<int *>(E.raw((size_t)Zw * 4));
    int *xsel = reinterpret_cast<int *>(E.raw((size_t)Zw * 4 * cols));
    double *amp = reinterpret_cast<double *>(E.raw((size_t)Zw * 16));
    int *kbuf = o.svd_cutoff > 0 ? reinterpret_cast<int *>(E.raw((size_t)Zw * 4 * std::max(cols - 1, 1))) : nullptr;
    std::vector<uint64_t> hidx(Zw);
    std::vector<int> hflags(Zw);
    // Per qubit, the outcome whose environment step runs for every sample: the
    // larger of |A[0]|^2 and |A[1]|^2 (a local guess at the likelier bit; the
    // other step runs masked for the samples that drew the other bit, so a
    // better guess means fewer unmasked tiles; results differ only in rounding)
    std::vector<int> favour((size_t)rows * cols, 0);
    {
        double *sn = reinterpret_cast<double *>(E.raw((size_t)rows * cols * 16));
        std::vector<double> hsn((size_t)rows * cols * 2, 0.0);
        for (int r = 0; r < rows; ++r)
            for (int c = 0; c < cols; ++c) {
                const SiteRef &a = V.at(r, c);
                if (a.dim(0) != 2) continue;
                const int64_t half = a.t->numel() / 2;
                E.norm2(a.t->p, a.t->esz, half, 2, half, sn + 2 * ((size_t)r * cols + c));
            }
        TN_HIP(hipMemcpyAsync(hsn.data(), sn, hsn.size() * 8, hipMemcpyDeviceToHost, E.s));
        E.sync();
        E.unraw(sn);
        for (size_t i = 0; i < favour.size(); ++i) favour[i] = hsn[2 * i + 1] > hsn[2 * i] ? 1 : 0;
    }
    // truncated (zero-padded) boundaries make the fit's QR inputs rank-deficient
    struct HouseholderScope {
        Engine &E;
        bool saved;
        HouseholderScope(Engine &e, bool on) : E(e), saved(e.householder_only) { E.householder_only = saved || on; }
        ~HouseholderScope() { E.householder_only = saved; }
    } hh(E, o.svd_cutoff > 0);
    // A wave reads and writes its samples through library buffers whose row 0
    // is the wave's first sample, so that its launch sequence does not depend
    // on the wave's position: the launches of the second full wave are captured
    // into a graph (the first one, run directly, creates the contraction plans
    // and tile choices) and replayed for the following full waves.
    const int nq = P.nq;
    double *u_w = uniforms ? reinterpret_cast<double *>(E.raw((size_t)Zw * nq * 8)) : nullptr;
    const int64_t bits_words = ((int64_t)Zw * nq + 3) / 4;  // cleared as int32 words
    uint8_t *bits_w = reinterpret_cast<uint8_t *>(E.raw((size_t)bits_words * 4));
    double *lq_w = reinterpret_cast<double *>(E.raw((size_t)Zw * 8));
    double *lp_w = log_p ? reinterpret_cast<double *>(E.raw((size_t)Zw * 8)) : nullptr;
    int *cu_w = chi_used ? reinterpret_cast<int *>(E.raw((size_t)Zw * rows * 4)) : nullptr;
    double *lc_w = o.log_cond ? reinterpret_cast<double *>(E.raw((size_t)Zw * nq * 8)) : nullptr;
    auto wave = [&](int Z, int64_t w0) {
        // bits of qubits that are not drawn (rows past a rows limit) read 0
        TN_HIP(tnk::launch_fill_i32(reinterpret_cast<int *>(bits_w), ((int64_t)Z * nq + 3) / 4, 0, E.s));
        TN_HIP(tnk::launch_fill_f64(mlog, Z, 0.0, E.s));
        TN_HIP(tnk::launch_fill_i32(flags, Z, 0, E.s));
        TN_HIP(tnk::launch_fill_f64(lq_w, Z, 0.0, E.s));
        std::vector<Ten> m(cols);
        for (int c = 0; c < cols; ++c) m[c] = ones(E, {Z, 1, V.at(0, c).dim(1), 1});
        if (cu_w) TN_HIP(tnk::launch_chi_used(nullptr, 0, Z, 1, cu_w, rows, E.s));
        const int rows_run = o.rows_limit > 0 ? std::min(rows, o.rows_limit) : rows;
        if (rows_run < rows && lp_w) TN_HIP(tnk::launch_fill_f64(lp_w, Z, NAN, E.s));
        for (int r = 0; r < rows_run; ++r) {
            const DMps &Bb = B.below[r];
            // sites that take the transfer-matrix route, and their matrices
            std::vector<int> useT(cols, 0);
            std::vector<Ten> Ts(cols), T0(cols), T1(cols);
            for (int c = 0; c < cols; ++c) {
                const SiteRef &a = V.at(r, c);
                if (!transfer_pays(a, Bb.site[c], m[c])) continue;
                useT[c] = 1;
                Ts[c] = transfer(E, a, Bb.site[c], -1);
                if (a.dim(0) == 2) {
                    T0[c] = transfer(E, a, Bb.site[c], 0);
                    T1[c] = transfer(E, a, Bb.site[c], 1);
                }
            }
            // Environments are rescaled to unit norm every ENV_RENORM sites only
            // (probabilities are ratios; the stride keeps them far from under-
            // and overflow).  R[c] is stored divided by exp(lnR[c][z]).
            std::vector<Ten> R(cols + 1);
            R[cols] = ones(E, {Z, 1, 1, 1, 1, 1});
            for (int c = cols - 1; c >= 1; --c) {
                R[c] = useT[c] ? env_right_T(E, R[c + 1], m[c], Ts[c])
                               : env_right(E, R[c + 1], m[c], V.at(r, c), Bb.site[c]);
                const int64_t per = R[c].numel() / Z;
                if ((cols - c) % ENV_RENORM == 0 || c == 1)
                    E.normalise(R[c].p, R[c].esz, per, Z, per, lnR + (size_t)c * Zw, false, nullptr);
                else
                    TN_HIP(tnk::launch_fill_f64(lnR + (size_t)c * Zw, Z, 0.0, E.s));
            }
            Ten Lc = ones(E, {Z, 1, 1, 1, 1, 1});
            for (int c = 0; c < cols; ++c) {
                const SiteRef &a = V.at(r, c);
                int *xs = xsel + (size_t)c * Zw;
                if (a.dim(0) == 1) {
                    Ten L2 = useT[c] ? env_left_T(E, Lc, m[c], Ts[c]) : env_left_traced(E, Lc, m[c], a, Bb.site[c]);
                    E.drop(Lc);
                    Lc = L2;
                    if ((c + 1) % ENV_RENORM == 0) unit(E, Lc, Z);
                    TN_HIP(tnk::launch_fill_i32(xs, Z, 0, E.s));
                    continue;
                }
                // P~(f) = <L_c . site(s=f), R_{c+1}> for the favoured bit f.  For
                // c >= 1 the traced right environment gives P~(0) + P~(1) =
                // |R_c| <L_c, R_c>, so the draw takes the other P~ as the
                // difference, except for samples where that difference is
                // below a precision-dependent fraction of the total (its
                // rounding would dominate): those contract the projection
                // directly before the draw.  After the draw the other bit's
                // step runs only for the samples that drew it (the others'
                // tiles are skipped), and their log q takes the conditional
                // from that direct projection.  Site 0 computes both.
                const int f = favour[(size_t)r * cols + c];
                auto rest_step = [&](const Ten &t1, int s) {
                    return useT[c] ? left_rest_T(E, t1, m[c], s ? T1[c] : T0[c])
                                   : left_rest(E, t1, m[c], a, Bb.site[c], s);
                };
                double *ptf = pt + (f ? 2 * Zw : 0), *pto = pt + (f ? 0 : 2 * Zw);
                Ten t1 = left_t1(E, Lc, m[c], useT[c] != 0);
                Ten Lf = rest_step(t1, f);
                const int64_t per = Lf.numel() / Z;
                E.dot(Lf.p, R[c + 1].p, Lf.esz, per, Z, per, ptf);
                Ten Lo;
                const bool rest = c >= 1;
                if (rest) {
                    const int64_t perc = Lc.numel() / Z;
                    E.dot(Lc.p, R[c].p, Lc.esz, perc, Z, perc, ptot);
                    TN_HIP(tnk::launch_marginal_rest(ptot, lnR + (size_t)c * Zw, ptf, pto, Z, diff_thr, need,
                                                     E.s));
                    // samples whose other-bit P~ is too small a difference to
                    // trust: contract that projection directly (masked to them)
                    E.set_mask(need, 'z', 0);
                    Ten Ln;
                    try {
                        Ln = rest_step(t1, 1 - f);
                    } catch (...) {
                        E.clear_mask();
                        throw;
                    }
                    E.clear_mask();
                    E.dot(Ln.p, R[c + 1].p, Ln.esz, per, Z, per, pto, need, 0);
                    E.drop(Ln);
                } else {
                    Lo = rest_step(t1, 1 - f);
                    E.dot(Lo.p, R[c + 1].p, Lo.esz, per, Z, per, pto);
                }
                tnk::DrawArgs d{};
                d.batch = Z;
                d.pt0 = pt;
                d.pt1 = pt + 2 * Zw;
                d.uniforms = u_w;
                d.u_row0 = 0;
                d.n_qubits = P.nq;
                d.qubit = P.site_index[(size_t)r * cols + c];
                d.seed = o.seed;
                d.sample_index = sidx;
                d.bits = bits_w;
                d.bits_row0 = 0;
                d.log_q = lq_w;
                d.xsel = xs;
                d.flags = flags;
                d.log_cond = lc_w;
                TN_HIP(tnk::launch_draw(d, E.s));
                if (rest) {
                    E.set_mask(xs, 'z', f);  // skip the samples that drew f
                    try {
                        Lo = rest_step(t1, 1 - f);
                    } catch (...) {
                        E.clear_mask();
                        throw;
                    }
                    E.clear_mask();
                    // the drawn bit's conditional from the direct projection
                    // (log q never keeps the difference's rounding)
                    E.dot(Lo.p, R[c + 1].p, Lo.esz, per, Z, per, ptd, xs, f);
                    TN_HIP(tnk::launch_fix_other(ptf, pto, ptd, xs, 1 - f, Z, lq_w, lc_w, 0, P.nq,
                                                 d.qubit, flags, E.s));
                }
                E.drop(t1);
                // keep the environment of the drawn bit: Lc[z] = (x_z ? L1 : L0)[z]
                const Ten &L0 = f ? Lo : Lf, &L1 = f ? Lf : Lo;
                E.drop(Lc);
                Lc = E.make(L0.d);
                TN_HIP(tnk::launch_select2(L0.p, L1.p, L0.esz, per, per, xs, Z, Lc.p, E.s));
                E.drop(Lf);
                E.drop(Lo);
                if ((c + 1) % ENV_RENORM == 0) unit(E, Lc, Z);
            }
            E.drop(Lc);
            for (auto &x : R)
                if (x.p) E.drop(x);
            for (int c = 0; c < cols; ++c)
                for (Ten *t : {&Ts[c], &T0[c], &T1[c]})
                    if (t->p) E.drop(*t);
            // projected row X_c[z] = A_c[x_c(z)], dims [z, u, h, d, H]
            std::vector<Ten> X(cols);
            for (int c = 0; c < cols; ++c) {
                const SiteRef &a = V.at(r, c);
                X[c] = E.make({Z, a.dim(1), a.dim(2), a.dim(3), a.dim(4)});
                const int64_t per = X[c].numel() / Z;
                TN_HIP(tnk::launch_select_copy(a.t->p, a.t->esz, per, per, 0, xsel + (size_t)c * Zw, Z, X[c].p,
                                               per, E.s));
            }
            if (r + 1 == rows_run && rows_run < rows) {
                // stopped early (test hook): no fit for rows that are not sampled
            } else if (r + 1 < rows) {
                std::vector<Ten> mn = fit_single(E, m, X, o, r, sidx, mlog);
                for (auto &x : m) E.drop(x);
                m = mn;
                if (o.svd_cutoff > 0) truncate_cutoff(E, m, o, kbuf);
                if (cu_w) {
                    int width = 1;
                    for (int c = 0; c + 1 < cols; ++c) width = std::max(width, m[c].d[3]);
                    TN_HIP(tnk::launch_chi_used(o.svd_cutoff > 0 ? kbuf : nullptr, cols - 1, Z, width,
                                                cu_w + r + 1, rows, E.s));
                }
            } else if (lp_w) {
                last_row_amplitude(E, m, X, mlog, amp, lp_w, nullptr);
            }
            for (auto &x : X) E.drop(x);
            if (progress_enabled()) {
                E.sync();
                std::fprintf(stderr, "tn: samples %lld-%lld row %d done\n", (long long)(first + w0),
                             (long long)(first + w0 + Z - 1), r);
                std::fflush(stderr);
            }
        }
        for (auto &x : m) E.drop(x);
    };
    Engine::Captured graph;
    bool have_graph = false;
    // per-launch event timing needs launches issued from the host: timed calls
    // (and progress reports, which synchronise per row) run every wave directly
    bool graphs_ok = o.graphs && !E.timing && !progress_enabled();
    int full_waves = 0;
    auto release_all = [&]() {
        if (have_graph) E.release(graph);
        have_graph = false;
        E.unraw(sidx); E.unraw(mlog); E.unraw(pt); E.unraw(flags); E.unraw(xsel); E.unraw(amp);
        E.unraw(ptot); E.unraw(lnR); E.unraw(ptd); E.unraw(need); E.unraw(bits_w); E.unraw(lq_w);
        for (void *q : {(void *)kbuf, (void *)u_w, (void *)lp_w, (void *)cu_w, (void *)lc_w})
            if (q) E.unraw(q);
    };
    try {
        for (int64_t w0 = 0; w0 < n; w0 += Zw) {
            const int Z = (int)std::min<int64_t>(Zw, n - w0);
            for (int z = 0; z < Z; ++z) hidx[z] = first + (uint64_t)(w0 + z);
            TN_HIP(hipMemcpyAsync(sidx, hidx.data(), (size_t)Z * 8, hipMemcpyHostToDevice, E.s));
            if (u_w)
                TN_HIP(hipMemcpyAsync(u_w, uniforms + w0 * nq, (size_t)Z * nq * 8, hipMemcpyDeviceToDevice, E.s));
            if (lc_w)
                TN_HIP(hipMemcpyAsync(lc_w, o.log_cond + w0 * nq, (size_t)Z * nq * 8, hipMemcpyDeviceToDevice, E.s));
            bool replayed = false;
            if (Z == Zw && graphs_ok && (have_graph || full_waves >= 1)) {
                if (!have_graph) {
                    bool ok = true;
                    try {
                        E.begin_capture(graph);
                    } catch (const TnError &) {
                        ok = false;
                    }
                    if (ok) {
                        try {
                            wave(Z, w0);
                        } catch (...) {
                            ok = false;
                        }
                        have_graph = E.end_capture(graph, ok);
                    }
                    if (!have_graph) graphs_ok = false;  // run this and later waves directly
                }
                if (have_graph) {
                    E.launch(graph);
                    replayed = true;
                } else {
                    wave(Z, w0);
                }
            } else {
                wave(Z, w0);
            }
            if (Z == Zw) ++full_waves;
            TN_HIP(hipMemcpyAsync(bits + w0 * nq, bits_w, (size_t)Z * nq, hipMemcpyDeviceToDevice, E.s));
            TN_HIP(hipMemcpyAsync(log_q + w0, lq_w, (size_t)Z * 8, hipMemcpyDeviceToDevice, E.s));
            if (lp_w) TN_HIP(hipMemcpyAsync(log_p + w0, lp_w, (size_t)Z * 8, hipMemcpyDeviceToDevice, E.s));
            if (cu_w)
                TN_HIP(hipMemcpyAsync(chi_used + w0 * rows, cu_w, (size_t)Z * rows * 4, hipMemcpyDeviceToDevice, E.s));
            if (lc_w)
                TN_HIP(hipMemcpyAsync(o.log_cond + w0 * nq, lc_w, (size_t)Z * nq * 8, hipMemcpyDeviceToDevice, E.s));
            TN_HIP(hipMemcpyAsync(hflags.data(), flags, (size_t)Z * 4, hipMemcpyDeviceToHost, E.s));
            E.sync();
            if (replayed && E.timing) E.collect_graph_timing(graph.pairs);
            for (int z = 0; z < Z; ++z)
                if (hflags[z])
                    throw TnError(ST_NUMERIC, "sample " + std::to_string(first + w0 + z) +
                                                  ((hflags[z] & 2) ? ": non-positive or non-finite marginal"
                                                                   : ": environment vanished or overflowed"));
        }
    } catch (...) {
        release_all();
        throw;
    }
    release_all();
}

void amplitude(Engine &E, const PepsDev &P, const SampleOpts &o, uint64_t first, int64_t n, const uint8_t *bits,
               double *log_p, double *arg) {
    const LView V = make_view(P, 0);
    const int rows = V.rows, cols = V.cols;
    int Zw = o.wave;
    if (Zw <= 0) {
        // peak per sample: the exact product m . X of one row and the fit's
        // intermediates, a few chi_x^2 D^3-sized tensors per site
        double per = 0;
        for (int r = 0; r < rows; ++r) {
            double row = 0;
            for (int c = 0; c < cols; ++c) {
                const SiteRef &a = V.at(r, c);
                const double x = o.chi_x;
                row += 6.0 * x * x * a.dim(1) * a.dim(2) * a.dim(3) * a.dim(4) / std::max(1, std::min(a.dim(1), a.dim(3)));
            }
            per = std::max(per, row);
        }
        per *= E.esz;
        size_t freeb = 0, total = 0;
        TN_HIP(hipMemGetInfo(&freeb, &total));
        const double budget = 0.5 * (double)freeb + 0.5 * (double)E.held();
        Zw = (int)std::max(1.0, std::min(4096.0, std::floor(budget / std::max(per, 1.0))));
    }
    Zw = (int)std::min<int64_t>(Zw, n);
    // the check contracts at a bond (typically 2 chi) well above the ranks of
    // the state's own bonds, where the fit's matrices are rank deficient:
    // Householder throughout instead of CholeskyQR with its per-item fallback
    struct HouseholderScope {
        Engine &E;
        bool saved;
        explicit HouseholderScope(Engine &e) : E(e), saved(e.householder_only) { E.householder_only = true; }
        ~HouseholderScope() { E.householder_only = saved; }
    } hh(E);
    uint64_t *sidx = reinterpret_cast<uint64_t *>(E.raw((size_t)Zw * 8));
    double *mlog = reinterpret_cast<double *>(E.raw((size_t)Zw * 8));
    int *xsel = reinterpret_cast<int *>(E.raw((size_t)Zw * 4 * cols));
    double *amp = reinterpret_cast<double *>(E.raw((size_t)Zw * 16));
    std::vector<uint64_t> hidx(Zw);
    try {
        for (int64_t w0 = 0; w0 < n; w0 += Zw) {
            const int Z = (int)std::min<int64_t>(Zw, n - w0);
            for (int z = 0; z < Z; ++z) hidx[z] = first + (uint64_t)(w0 + z);
            TN_HIP(hipMemcpyAsync(sidx, hidx.data(), (size_t)Z * 8, hipMemcpyHostToDevice, E.s));
            TN_HIP(tnk::launch_fill_f64(mlog, Z, 0.0, E.s));
            std::vector<Ten> m(cols);
            for (int c = 0; c < cols; ++c) m[c] = ones(E, {Z, 1, V.at(0, c).dim(1), 1});
            for (int r = 0; r < rows; ++r) {
                std::vector<Ten> X(cols);
                for (int c = 0; c < cols; ++c) {
                    const SiteRef &a = V.at(r, c);
                    int *xs = xsel + (size_t)c * Zw;
                    const int q = P.site_index[(size_t)r * cols + c];
                    if (a.dim(0) == 1 || q < 0) TN_HIP(tnk::launch_fill_i32(xs, Z, 0, E.s));
                    else TN_HIP(tnk::launch_bits_select(bits, P.nq, w0, q, Z, xs, E.s));
                    X[c] = E.make({Z, a.dim(1), a.dim(2), a.dim(3), a.dim(4)});
                    const int64_t per = X[c].numel() / Z;
                    TN_HIP(tnk::launch_select_copy(a.t->p, a.t->esz, per, per, 0, xs, Z, X[c].p, per, E.s));
                }
                if (r + 1 < rows) {
                    std::vector<Ten> mn = fit_single(E, m, X, o, r, sidx, mlog);
                    for (auto &x : m) E.drop(x);
                    m = mn;
                } else {
                    last_row_amplitude(E, m, X, mlog, amp, log_p + w0, arg ? arg + w0 : nullptr);
                }
                for (auto &x : X) E.drop(x);
            }
            for (auto &x : m) E.drop(x);
        }
    } catch (...) {
        E.unraw(sidx); E.unraw(mlog); E.unraw(xsel); E.unraw(amp);
        throw;
    }
    E.unraw(sidx); E.unraw(mlog); E.unraw(xsel); E.unraw(amp);
}

}  // namespace tnb
