// Boundary MPSs through the rows of the norm network <psi|psi>, each MPS-MPO
// product compressed by the one-site variational fit (Methods, "The Boundary
// Matrix Product State Method"; Appendix, "Sampling from a Tensor Network
// State", Fig. 7c: the fit replaces each site of the output MPS by the
// derivative of the MPS-MPO-MPS overlap with respect to it).
//
// Ket and bra tensors of a row are never fused: every contraction takes the
// row tensor A and its conjugate separately.  Readings where the paper is
// silent: an exactly representable product is applied exactly and brought to
// canonical form by QR sweeps; otherwise the initial guess is a Philox-uniform
// MPS with the target bonds, right-canonicalised by LQ; a sweep is QR
// left-to-right then LQ right-to-left; the centre ends on site 0 and is
// normalised into a log-scale.
#include "tn_core.hpp"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cmath>

namespace tnb {

// ---------------------------------------------------------------- views

LView make_view(const PepsDev &P, int direction) {
    LView V;
    const bool tr = (direction == 2 || direction == 3);
    const bool flip = (direction == 1 || direction == 3);
    V.rows = tr ? P.cols : P.rows;
    V.cols = tr ? P.rows : P.cols;
    V.s.resize((size_t)V.rows * V.cols);
    for (int r = 0; r < V.rows; ++r)
        for (int c = 0; c < V.cols; ++c) {
            const int r1 = flip ? V.rows - 1 - r : r;  // row in the (possibly transposed) lattice
            const int orow = tr ? c : r1, ocol = tr ? r1 : c;
            SiteRef a;
            a.t = &P.at(orow, ocol);
            int p1[5] = {0, 1, 2, 3, 4};
            if (tr) { int q[5] = {0, 2, 1, 4, 3}; std::copy(q, q + 5, p1); }
            if (flip) {
                // view (s,u,l,d,r) = mirrored (s,d,l,u,r) of the transposed lattice
                int q[5] = {p1[0], p1[3], p1[2], p1[1], p1[4]};
                std::copy(q, q + 5, p1);
            }
            std::copy(p1, p1 + 5, a.perm);
            V.s[(size_t)r * V.cols + c] = a;
        }
    return V;
}

static void strides5(const Ten &t, int64_t st[5]) {
    st[4] = 1;
    for (int i = 3; i >= 0; --i) st[i] = st[i + 1] * t.d[i + 1];
}

Op sop(const SiteRef &a, const std::string &L, bool conj) {
    int64_t st[5];
    strides5(*a.t, st);
    Op o;
    o.p = a.t->p;
    o.esz = a.t->esz;
    o.idx = L;
    o.conj = conj;
    for (int i = 0; i < 5; ++i) {
        o.dims.push_back(a.t->d[a.perm[i]]);
        o.str.push_back(st[a.perm[i]]);
    }
    return o;
}

Op sop_proj(const SiteRef &a, int s, const std::string &L, bool conj) {
    int64_t st[5];
    strides5(*a.t, st);
    Op o;
    o.esz = a.t->esz;
    o.p = reinterpret_cast<const char *>(a.t->p) + (int64_t)s * st[a.perm[0]] * a.t->esz;
    o.idx = L;
    o.conj = conj;
    for (int i = 1; i < 5; ++i) {
        o.dims.push_back(a.t->d[a.perm[i]]);
        o.str.push_back(st[a.perm[i]]);
    }
    return o;
}

// ---------------------------------------------------------------- helpers

// TN_PROGRESS=1 in the environment: long loops wait for each row and report it
// on stderr (for runs whose single calls take minutes).
bool progress_enabled() {
    const char *v = std::getenv("TN_PROGRESS");
    return v && v[0] == '1';
}

Ten ones(Engine &E, const std::vector<int> &dims) {
    Ten t = E.make(dims);
    TN_HIP(tnk::launch_fill(t.p, t.esz, t.numel(), 1.0, 0.0, E.s));
    return t;
}

static int64_t prod(const std::vector<int> &d, int a, int b) {
    int64_t p = 1;
    for (int i = a; i < b; ++i) p *= d[i];
    return p;
}

// QR of T seen as batch x m x n (batch = first nb dims, n = last dim).
// well_conditioned: R may come from CholeskyQR3 (see Engine::orthonormalise).
void qr_left(Engine &E, const Ten &T, int nb, Ten &Q, Ten *R, bool well_conditioned) {
    const int rk = (int)T.d.size();
    const int64_t batch = prod(T.d, 0, nb);
    const int64_t n = T.d[rk - 1];
    const int64_t m = prod(T.d, nb, rk - 1);
    const int64_t k = std::min(m, n);
    std::vector<int> qd = T.d;
    qd[rk - 1] = (int)k;
    Q = E.make(qd, T.esz);
    if (R) {
        std::vector<int> rd(T.d.begin(), T.d.begin() + nb);
        rd.push_back((int)k);
        rd.push_back((int)n);
        *R = E.make(rd, T.esz);
    }
    if (m == n) {
        // a square factor spans the whole space: Q = I, R = T is an exact
        // factorisation in another gauge (every output is gauge invariant)
        TN_HIP(tnk::launch_eye(Q.p, Q.esz, (int)n, (int)batch, E.s));
        if (R) TN_HIP(tnk::launch_convert(T.p, T.esz, R->p, R->esz, T.numel(), E.s));
        return;
    }
    tnk::QrArgs a{};
    a.m = (int)m; a.n = (int)n; a.batch = (int)batch;
    a.A = T.p; a.a_esz = T.esz; a.a_bs = m * n; a.a_rs = n; a.a_cs = 1; a.a_conj = 0;
    a.Q = Q.p; a.q_esz = Q.esz; a.q_bs = m * k; a.q_rs = k; a.q_cs = 1; a.q_conj = 0;
    a.R = R ? R->p : nullptr; a.r_esz = T.esz; a.r_bs = k * n; a.r_rs = n; a.r_cs = 1; a.r_conj = 0;
    // the fit needs only an orthonormal basis of the column space
    if (R && !well_conditioned) E.qr(a);
    else E.orthonormalise(a);
}

// LQ of T seen as batch x m x n (m = dim nb, n = the rest): T = L Q, Q rows orthonormal.
void lq_right(Engine &E, const Ten &T, int nb, Ten &Q, Ten *Lf, bool well_conditioned) {
    const int rk = (int)T.d.size();
    const int64_t batch = prod(T.d, 0, nb);
    const int64_t m = T.d[nb];
    const int64_t n = prod(T.d, nb + 1, rk);
    const int64_t k = std::min(m, n);
    std::vector<int> qd = T.d;
    qd[nb] = (int)k;
    Q = E.make(qd, T.esz);
    if (Lf) {
        std::vector<int> ld(T.d.begin(), T.d.begin() + nb);
        ld.push_back((int)m);
        ld.push_back((int)k);
        *Lf = E.make(ld, T.esz);
    }
    if (m == n) {  // square: Q = I, L = T (see qr_left)
        TN_HIP(tnk::launch_eye(Q.p, Q.esz, (int)n, (int)batch, E.s));
        if (Lf) TN_HIP(tnk::launch_convert(T.p, T.esz, Lf->p, Lf->esz, T.numel(), E.s));
        return;
    }
    // QR of T^H (n x m): T^H(i, j) = conj(T[j][i])
    tnk::QrArgs a{};
    a.m = (int)n; a.n = (int)m; a.batch = (int)batch;
    a.A = T.p; a.a_esz = T.esz; a.a_bs = m * n; a.a_rs = 1; a.a_cs = n; a.a_conj = 1;
    a.Q = Q.p; a.q_esz = Q.esz; a.q_bs = k * n; a.q_rs = 1; a.q_cs = n; a.q_conj = 1;
    a.R = Lf ? Lf->p : nullptr; a.r_esz = T.esz; a.r_bs = m * k; a.r_rs = 1; a.r_cs = k; a.r_conj = 1;
    if (Lf && !well_conditioned) E.qr(a);
    else E.orthonormalise(a);
}

void plan_bonds(const std::vector<int> &phys, const std::vector<int64_t> &bond_in, int chi,
                bool &exact_ok, std::vector<int> &t) {
    const int L = (int)phys.size();
    std::vector<int64_t> ex(std::max(L - 1, 0));
    for (int c = 0; c + 1 < L; ++c) {
        // products saturate: only comparisons with chi and bond_in matter
        int64_t pl = 1, pr = 1;
        for (int i = 0; i <= c; ++i) pl = std::min<int64_t>(pl * phys[i], (int64_t)1 << 40);
        for (int i = c + 1; i < L; ++i) pr = std::min<int64_t>(pr * phys[i], (int64_t)1 << 40);
        ex[c] = std::min(std::min(pl, pr), bond_in[c]);
    }
    // exact when chi reaches the bound at every cut and the exact product is
    // small (its bond <= max(chi, 64)); a row with few sites can have a small
    // bound but a huge product bond, which is fitted to the bound instead
    exact_ok = true;
    for (int64_t e : ex)
        if ((int64_t)chi < e) exact_ok = false;
    for (int64_t b : bond_in)
        if (b > std::max<int64_t>(chi, 64)) exact_ok = false;
    t.assign(std::max(L - 1, 0), 0);
    for (int c = 0; c + 1 < L; ++c) t[c] = (int)std::min<int64_t>(chi, ex[c]);
    for (int c = 0; c + 1 < L; ++c) {
        const int64_t left = c > 0 ? t[c - 1] : 1;
        t[c] = (int)std::min<int64_t>(t[c], left * phys[c]);
    }
    for (int c = L - 2; c >= 0; --c) {
        const int64_t right = c < L - 2 ? t[c + 1] : 1;
        t[c] = (int)std::min<int64_t>(t[c], (int64_t)phys[c + 1] * right);
    }
}

void free_mps(Engine &E, DMps &m) {
    for (auto &t : m.site)
        if (t.p) E.drop(t);
    m.site.clear();
}

void free_set(Engine &E, BoundarySet &b) {
    for (auto &m : b.below) free_mps(E, m);
    b.below.clear();
    if (b.logs) E.unraw(b.logs);
    b.logs = nullptr;
}

// Canonical form by QR sweeps (no truncation); nb = number of leading batch dims
// (0: double-layer sites [yl][u][v][yr]; 1: batched single-layer [z][a][d][A]).
void canonicalise(Engine &E, std::vector<Ten> &Y, int nb, double *logscale, bool acc) {
    const int L = (int)Y.size();
    for (int c = 0; c + 1 < L; ++c) {
        Ten Q, R;
        qr_left(E, Y[c], nb, Q, &R);
        E.drop(Y[c]);
        Y[c] = Q;
        Ten N = nb ? E.contract_new(op(R, "zab"), op(Y[c + 1], "zbcd"), "zacd")
                   : E.contract_new(op(R, "ab"), op(Y[c + 1], "bcde"), "acde");
        E.drop(R);
        E.drop(Y[c + 1]);
        Y[c + 1] = N;
    }
    for (int c = L - 1; c >= 1; --c) {
        Ten Q, Lm;
        lq_right(E, Y[c], nb, Q, &Lm);
        E.drop(Y[c]);
        Y[c] = Q;
        Ten N = nb ? E.contract_new(op(Y[c - 1], "zabc"), op(Lm, "zcd"), "zabd")
                   : E.contract_new(op(Y[c - 1], "abcd"), op(Lm, "de"), "abce");
        E.drop(Lm);
        E.drop(Y[c - 1]);
        Y[c - 1] = N;
    }
    const int batch = nb ? Y[0].d[0] : 1;
    const int64_t per = Y[0].numel() / batch;
    E.normalise(Y[0].p, Y[0].esz, per, batch, per, logscale, acc, nullptr);
}

// Right-canonicalise a (batched) MPS by LQ sweeps from the right.  Used on the
// fits' random initial guesses, whose factors are well conditioned.
void right_canonicalise(Engine &E, std::vector<Ten> &Y, int nb) {
    const int L = (int)Y.size();
    for (int c = L - 1; c >= 1; --c) {
        Ten Q, Lm;
        lq_right(E, Y[c], nb, Q, &Lm, true);
        E.drop(Y[c]);
        Y[c] = Q;
        Ten N = nb ? E.contract_new(op(Y[c - 1], "zabc"), op(Lm, "zcd"), "zabd")
                   : E.contract_new(op(Y[c - 1], "abcd"), op(Lm, "de"), "abce");
        E.drop(Lm);
        E.drop(Y[c - 1]);
        Y[c - 1] = N;
    }
}

// t[y,G,u,H,v,K] = sum L[y,g,h,k] B[g,d,e,G] A[s,u,h,d,H] conj(A)[s,v,k,e,K]
static Ten left_partial(Engine &E, const Ten &Le, const Ten &B, const SiteRef &a) {
    Ten t1 = E.contract_new(op(Le, "yghk"), op(B, "gdeG"), "yhkdeG");
    Ten t2 = E.contract_new(op(t1, "yhkdeG"), sop(a, "suhdH"), "ykeGsuH");
    E.drop(t1);
    Ten t3 = E.contract_new(op(t2, "ykeGsuH"), sop(a, "svkeK", true), "yGuHvK");
    E.drop(t2);
    return t3;
}

// t[g,Y,u,h,v,k] = sum B[g,d,e,G] A[s,u,h,d,H] conj(A)[s,v,k,e,K] R[Y,G,H,K]
// (the letters of t2 keep their order in t, h innermost, as in t2, so that the
// last product streams t2 along its contiguous letter)
static Ten right_partial(Engine &E, const Ten &Re, const Ten &B, const SiteRef &a) {
    Ten t1 = E.contract_new(op(B, "gdeG"), op(Re, "YGHK"), "gdeYHK");
    Ten t2 = E.contract_new(op(t1, "gdeYHK"), sop(a, "suhdH"), "geYKsuh");
    E.drop(t1);
    Ten t3 = E.contract_new(op(t2, "geYKsuh"), sop(a, "svkeK", true), "gYuhvk");
    E.drop(t2);
    return t3;
}

static DMps fit_double(Engine &E, const DMps &Bin, const LView &V, int r, const FitOpts &o, uint64_t tag,
                       double *logscale, int *mode) {
    const int L = V.cols;
    std::vector<int> phys(L);
    std::vector<int64_t> bin(std::max(L - 1, 0));
    for (int c = 0; c < L; ++c) phys[c] = V.at(r, c).dim(1) * V.at(r, c).dim(1);
    for (int c = 0; c + 1 < L; ++c)
        bin[c] = (int64_t)Bin.site[c].d[3] * V.at(r, c).dim(4) * V.at(r, c).dim(4);
    bool exact;
    std::vector<int> t;
    plan_bonds(phys, bin, o.chi, exact, t);
    DMps Y;
    Y.site.resize(L);
    if (exact && !o.force_fit) {
        *mode = 1;
        for (int c = 0; c < L; ++c) {
            const Ten &B = Bin.site[c];
            const SiteRef &a = V.at(r, c);
            Ten X = E.contract_new(op(B, "gdeG"), sop(a, "suhdH"), "geGsuhH");
            Ten Yc = E.contract_new(op(X, "geGsuhH"), sop(a, "svkeK", true), "ghkuvGHK");
            E.drop(X);
            const int h = a.dim(2), H = a.dim(4), u = a.dim(1);
            Yc.d = {B.d[0] * h * h, u, u, B.d[3] * H * H};
            Y.site[c] = Yc;
        }
        canonicalise(E, Y.site, 0, logscale, false);
        return Y;
    }
    *mode = 2;
    for (int c = 0; c < L; ++c) {
        const int tl = c > 0 ? t[c - 1] : 1, tr = c + 1 < L ? t[c] : 1, u = V.at(r, c).dim(1);
        Y.site[c] = E.make({tl, u, u, tr});
        TN_HIP(tnk::launch_init_tensor(Y.site[c].p, Y.site[c].esz, Y.site[c].numel(), 1, 0, o.seed, tag,
                                       (uint64_t)r, (uint64_t)c, nullptr, E.s));
    }
    right_canonicalise(E, Y.site, 0);
    std::vector<Ten> Le(L + 1), Re(L + 1);
    Re[L] = ones(E, {1, 1, 1, 1});
    Le[0] = ones(E, {1, 1, 1, 1});
    for (int c = L - 1; c >= 1; --c) {
        Ten tR = right_partial(E, Re[c + 1], Bin.site[c], V.at(r, c));
        Re[c] = E.contract_new(op(Y.site[c], "yuvY", true), op(tR, "gYuhvk"), "yghk");
        E.drop(tR);
    }
    for (int sw = 0; sw < o.sweeps; ++sw) {
        for (int c = 0; c + 1 < L; ++c) {
            Ten t3 = left_partial(E, Le[c], Bin.site[c], V.at(r, c));
            Ten N = E.contract_new(op(t3, "yGuHvK"), op(Re[c + 1], "YGHK"), "yuvY");
            Ten Q;
            qr_left(E, N, 0, Q, nullptr);
            E.drop(N);
            E.drop(Y.site[c]);
            Y.site[c] = Q;
            if (Le[c + 1].p) E.drop(Le[c + 1]);
            Le[c + 1] = E.contract_new(op(Y.site[c], "yuvY", true), op(t3, "yGuHvK"), "YGHK");
            E.drop(t3);
        }
        for (int c = L - 1; c >= 1; --c) {
            Ten tR = right_partial(E, Re[c + 1], Bin.site[c], V.at(r, c));
            Ten N = E.contract_new(op(Le[c], "yghk"), op(tR, "gYuhvk"), "yuvY");
            Ten Q;
            lq_right(E, N, 0, Q, nullptr);
            E.drop(N);
            E.drop(Y.site[c]);
            Y.site[c] = Q;
            if (Re[c].p) E.drop(Re[c]);
            Re[c] = E.contract_new(op(Y.site[c], "yuvY", true), op(tR, "gYuhvk"), "yghk");
            E.drop(tR);
        }
    }
    {
        Ten tR = right_partial(E, Re[1], Bin.site[0], V.at(r, 0));
        Ten N = E.contract_new(op(Le[0], "yghk"), op(tR, "gYuhvk"), "yuvY");
        E.drop(tR);
        E.drop(Y.site[0]);
        Y.site[0] = N;
    }
    for (auto &x : Le)
        if (x.p) E.drop(x);
    for (auto &x : Re)
        if (x.p) E.drop(x);
    E.normalise(Y.site[0].p, Y.site[0].esz, Y.site[0].numel(), 1, 0, logscale, false, nullptr);
    return Y;
}

BoundarySet boundary_set(Engine &E, const LView &V, const FitOpts &o, uint64_t tag) {
    BoundarySet S;
    S.rows = V.rows;
    S.below.resize(V.rows);
    S.mode.assign(V.rows, 0);
    S.logs = reinterpret_cast<double *>(E.raw((size_t)V.rows * 8));
    TN_HIP(tnk::launch_fill_f64(S.logs, V.rows, 0.0, E.s));
    DMps &last = S.below[V.rows - 1];
    for (int c = 0; c < V.cols; ++c) {
        const int d = V.at(V.rows - 1, c).dim(3);
        last.site.push_back(ones(E, {1, d, d, 1}));
    }
    const bool progress = progress_enabled();
    for (int r = V.rows - 1; r >= 1; --r) {
        S.below[r - 1] = fit_double(E, S.below[r], V, r, o, tag, S.logs + (r - 1), &S.mode[r - 1]);
        if (progress) {
            E.sync();
            std::fprintf(stderr, "tn: boundary below row %d done\n", r - 1);
            std::fflush(stderr);
        }
    }
    return S;
}

void norm_close(Engine &E, const LView &V, const BoundarySet &B, double *logabs, double *arg) {
    Ten Le = ones(E, {1, 1, 1, 1});
    double *lg = reinterpret_cast<double *>(E.raw(8));
    TN_HIP(tnk::launch_fill_f64(lg, 1, 0.0, E.s));
    for (int c = 0; c < V.cols; ++c) {
        Ten t3 = left_partial(E, Le, B.below[0].site[c], V.at(0, c));  // [y,G,u,H,v,K], y=u=v=1
        E.drop(Le);
        Le = t3;
        Le.d = {t3.d[0] * t3.d[2] * t3.d[4], t3.d[1], t3.d[3], t3.d[5]};
        // keep the running product in range (FP32 modes); the scale goes to lg
        E.normalise(Le.p, Le.esz, Le.numel(), 1, 0, lg, true, nullptr);
    }
    // after the last site Le is a unit-modulus scalar
    double z[2] = {0, 0};
    if (Le.esz == 16) {
        TN_HIP(hipMemcpyAsync(z, Le.p, 16, hipMemcpyDeviceToHost, E.s));
    } else {
        float f[2];
        TN_HIP(hipMemcpyAsync(f, Le.p, 8, hipMemcpyDeviceToHost, E.s));
        E.sync();
        z[0] = f[0]; z[1] = f[1];
    }
    std::vector<double> logs(B.rows);
    double lgh = 0;
    TN_HIP(hipMemcpyAsync(logs.data(), B.logs, (size_t)B.rows * 8, hipMemcpyDeviceToHost, E.s));
    TN_HIP(hipMemcpyAsync(&lgh, lg, 8, hipMemcpyDeviceToHost, E.s));
    E.sync();
    E.drop(Le);
    E.unraw(lg);
    double s = lgh;
    for (double x : logs) s += x;
    const double a = std::hypot(z[0], z[1]);
    if (!(a > 0.0) || !std::isfinite(a) || !std::isfinite(s))
        throw TnError(ST_NUMERIC, "norm contraction vanished or overflowed");
    *logabs = s + std::log(a);
    *arg = std::atan2(z[1], z[0]);
}

}  // namespace tnb
