// Circuit simulation by BP-gauged simple update (Methods, "Quantum Circuit
// Simulation": each two-qubit gate applied to its pair of site tensors and the
// shared bond truncated back by an SVD, the pair's environment replaced by the
// BP messages of the norm network, refreshed between groups of gates that share
// no qubit; the gate error of Eq. error_per_gate and the fidelity estimate of
// Eq. total_fidelity.  Appendix, "Applying Gates to a Tensor Network State":
// gauge with the square roots of the incoming messages, apply, SVD, ungauge
// with their inverses).
//
// FP64 throughout.  Per group: BP messages (bp_contract, started from the
// previous group's converged messages), then the square root
// and its pseudo-inverse of every message from one batched SVD (a Hermitian
// positive message has U = V; values at or below 1e-12 of the largest are
// dropped, which makes the inverse a pseudo-inverse).  Per gate (site v, site w
// sharing bond b of dimension D):
//   1. gauge the three other legs of v and of w with the message roots, the
//      last contraction ordering each tensor as [other legs][phys][b];
//   2. reduce: QR of v as (other legs) x (phys, b) and of w likewise (the SVD
//      of the pair equals that of R_v R_w^T up to the isometries Q);
//   3. theta[(i s'), (j t')] = sum G[s' t', s t] R_v[i, s, b] R_w[j, t, b],
//      normalised, zero-padded to a square of side n = max(2 k_v, 2 k_w, D);
//   4. SVD truncated to min(D, rank) values; eps = discarded weight;
//      U S^{1/2} and S^{1/2} V^H back through Q_v and Q_w;
//   5. ungauge with the pseudo-inverse roots, the last contraction writing the
//      site tensor in its own layout [p][u][l][d][r].
#include "tn_core.hpp"

#include <algorithm>
#include <cmath>

namespace tnb {

namespace {

const char SLOT[5] = {'s', 'u', 'l', 'd', 'r'};   // site tensor letters
const char GAUGED[5] = {'S', 'U', 'L', 'D', 'R'};  // the same legs after gauging

Op raw_op(const void *p, const std::string &idx, std::vector<int> dims, std::vector<int64_t> str) {
    Op o;
    o.p = p;
    o.esz = 16;
    o.idx = idx;
    o.dims = std::move(dims);
    o.str = std::move(str);
    return o;
}

// The D_x x D_x block of a padded [z][leg][Dm][Dm] root array for slot x (1..4)
// of site z, with letters (row, column).
Op root_op(const Ten &roots, int z, int slot, int Dx, int Dm, char row, char col) {
    const char *p = static_cast<const char *>(roots.p) + (((size_t)z * 4 + (slot - 1)) * Dm * Dm) * 16;
    return raw_op(p, std::string{row, col}, {Dx, Dx}, {Dm, 1});
}

// Letters of a site tensor after gauging the legs in `done` (uppercase).
std::string letters(const bool done[5]) {
    std::string s;
    for (int k = 0; k < 5; ++k) s.push_back(done[k] ? GAUGED[k] : SLOT[k]);
    return s;
}

// Gauge the three legs of site z other than `bond` with the message roots:
// returns a tensor ordered [G1][G2][G3][s][b] (G = gauged leg letters, in slot
// order), the bond leg b = SLOT[bond].
Ten gauge_site(Engine &E, const Ten &A, const Ten &Sq, int z, int bond, int Dm, std::string &ext) {
    bool done[5] = {false, false, false, false, false};
    ext.clear();
    for (int k = 1; k <= 4; ++k)
        if (k != bond) ext.push_back(GAUGED[k]);
    Ten cur;
    bool have = false;
    int count = 0;
    for (int k = 1; k <= 4; ++k) {
        if (k == bond) continue;
        ++count;
        const std::string in = letters(done);
        done[k] = true;
        std::string out = letters(done);
        if (count == 3) out = ext + std::string{SLOT[0], SLOT[bond]};
        const Op src = have ? op(cur, in) : op(A, in);
        Ten nxt = E.contract_new(src, root_op(Sq, z, k, A.d[k], Dm, SLOT[k], GAUGED[k]), out);
        if (have) E.drop(cur);
        cur = nxt;
        have = true;
    }
    return cur;
}

// Undo the gauge: T ordered `in` (gauged legs uppercase), the pseudo-inverse
// roots applied leg by leg, the last product written into the site tensor.
void ungauge_site(Engine &E, const Ten &T, const std::string &in, const Ten &Sp, int z, const Ten &site, int bond,
                  int Dm) {
    Ten cur;
    bool have = false;
    std::string cin = in;
    int count = 0;
    for (int k = 1; k <= 4; ++k) {
        if (k == bond) continue;
        ++count;
        std::string out = cin;
        out[out.find(GAUGED[k])] = SLOT[k];
        const Op src = have ? op(cur, cin) : op(T, cin);
        const Op R = root_op(Sp, z, k, site.d[k], Dm, GAUGED[k], SLOT[k]);
        if (count == 3) {
            E.contract(src, R, op(site, "suldr"));
        } else {
            Ten nxt = E.contract_new(src, R, out);
            if (have) E.drop(cur);
            cur = nxt;
            have = true;
        }
        cin = out;
    }
    if (have) E.drop(cur);
}

}  // namespace

void simple_update(Engine &E, PepsDev &P, const std::vector<SuGate> &gates, const double *gmat, int gstride,
                   const SuOpts &o, double *eps_host) {
    const int rows = P.rows, cols = P.cols, N = rows * cols;
    const int ng = (int)gates.size();
    if (ng == 0) return;
    int Dm = 1;
    for (const Ten &t : P.site)
        for (int k = 1; k <= 4; ++k) Dm = std::max(Dm, t.d[k]);
    if (Dm > 32) throw TnError(ST_UNSUPPORTED, "simple update: bonds above 32 (the pair SVD is at most 128 wide)");
    // gate matrices on the device: one per gate (gstride 16) or one for all (0)
    const int nmat = gstride ? ng : 1;
    Ten Gd = E.make({nmat, 4, 4});
    Ten msg = E.make({N, 4, Dm, Dm});
    Ten Um = E.make({N * 4, Dm, Dm}), SVm = E.make({N * 4, Dm, Dm});
    Ten Sq = E.make({N * 4, Dm, Dm}), Sp = E.make({N * 4, Dm, Dm});
    int *kmsg = static_cast<int *>(E.raw((size_t)N * 4 * sizeof(int)));
    double *eps_d = static_cast<double *>(E.raw((size_t)ng * sizeof(double)));
    const int nmax = 4 * Dm;  // largest padded theta side (k <= 2 D per side, D <= Dm)
    Ten M = E.make({nmax * nmax});
    Ten Uv = E.make({nmax * nmax}), SVv = E.make({nmax * nmax});
    int *kg = static_cast<int *>(E.raw(sizeof(int)));
    void *svd_ws = nullptr;
    const size_t wsb = std::max(tnk::svd_trunc_workspace_bytes(nmax, 1), tnk::svd_trunc_workspace_bytes(Dm, N * 4));
    if (wsb) svd_ws = E.raw(wsb);
    auto cleanup = [&]() {
        E.drop(Gd); E.drop(msg); E.drop(Um); E.drop(SVm); E.drop(Sq); E.drop(Sp);
        E.drop(M); E.drop(Uv); E.drop(SVv);
        E.unraw(kmsg); E.unraw(eps_d); E.unraw(kg);
        if (svd_ws) E.unraw(svd_ws);
    };
    try {
        TN_HIP(hipMemcpyAsync(Gd.p, gmat, (size_t)nmat * 16 * 16, hipMemcpyHostToDevice, E.s));
        int cur_group = 0;
        bool first = true;
        for (int g = 0; g < ng; ++g) {
            const SuGate &q = gates[g];
            if (first || q.group != cur_group) {
                BpOpts bo;
                bo.max_sweeps = o.bp_max_sweeps;
                bo.tol = o.bp_tol;
                bo.loops = false;
                bo.messages = msg.p;
                bo.init_messages = first ? nullptr : msg.p;  // warm start from the previous group's messages
                BpResult br;
                bp_contract(E, P, bo, br);
                TN_HIP(tnk::launch_svd_trunc(static_cast<const double *>(msg.p), Dm, N * 4, 0.0, 0, Um.p, SVm.p, 16,
                                             kmsg, svd_ws, E.s));
                TN_HIP(tnk::launch_msg_roots(static_cast<const double *>(Um.p), static_cast<const double *>(SVm.p),
                                             Dm, N * 4, static_cast<double *>(Sq.p), static_cast<double *>(Sp.p),
                                             E.s));
                cur_group = q.group;
                first = false;
            }
            const bool horiz = q.r2 == q.r;
            const int lv = horiz ? 4 : 3, lw = horiz ? 2 : 1;
            const int zv = q.r * cols + q.c, zw = q.r2 * cols + q.c2;
            const Ten &A = P.site[zv], &B = P.site[zw];
            const int Db = A.d[lv];
            // 1. gauge, ordered [other legs][phys][bond]
            std::string ev, ew;
            Ten Ag = gauge_site(E, A, Sq, zv, lv, Dm, ev);
            Ten Bg = gauge_site(E, B, Sq, zw, lw, Dm, ew);
            // 2. QR of (other legs) x (phys, bond)
            const std::vector<int> agd = Ag.d, bgd = Bg.d;
            Ag.d = {agd[0], agd[1], agd[2], agd[3] * agd[4]};
            Bg.d = {bgd[0], bgd[1], bgd[2], bgd[3] * bgd[4]};
            Ten QA, RA, QB, RB;
            qr_left(E, Ag, 0, QA, &RA);
            qr_left(E, Bg, 0, QB, &RB);
            E.drop(Ag);
            E.drop(Bg);
            const int kA = RA.d[0], kB = RB.d[0];
            RA.d = {kA, 2, Db};
            RB.d = {kB, 2, Db};
            // 3. theta through the gate, into the zero-padded square
            // square side: both factors' rows and the bond's D columns fit in it
            const int n = std::max(std::max(2 * kA, 2 * kB), Db);
            Ten T1 = E.contract_new(op(RA, "isb"), op(RB, "jtb"), "isjt");
            E.drop(RA);
            E.drop(RB);
            TN_HIP(tnk::launch_fill(M.p, 16, (int64_t)n * n, 0.0, 0.0, E.s));
            const char *gp = static_cast<const char *>(Gd.p) + (size_t)(gstride ? g : 0) * 16 * 16;
            E.contract(op(T1, "isjt"), raw_op(gp, "STst", {2, 2, 2, 2}, {8, 4, 2, 1}),
                       raw_op(M.p, "iSjT", {kA, 2, kB, 2}, {2LL * n, n, 2, 1}));
            E.drop(T1);
            E.normalise(M.p, 16, (int64_t)n * n, 1, 0, nullptr, false, nullptr);
            // 4. truncated SVD, balanced factors
            TN_HIP(tnk::launch_svd_trunc(static_cast<const double *>(M.p), n, 1, 0.0, 0, Uv.p, SVv.p, 16, kg, svd_ws,
                                         E.s, Db, eps_d + g));
            TN_HIP(tnk::launch_split_sqrt(static_cast<double *>(Uv.p), static_cast<double *>(SVv.p), n, 1, E.s));
            const char bv = SLOT[lv], bw = SLOT[lw];
            // v: [ev][s][b] = sum_i Q_A[ev][i] U[(i s)][b]
            Ten An = E.contract_new(op(QA, ev + "i"), raw_op(Uv.p, std::string{'i', 's', bv}, {kA, 2, Db}, {2LL * n, n, 1}),
                                    ev + std::string{'s', bv});
            // w: [ew][t][b] = sum_j SV[b][(j t)] Q_B[ew][j]
            Ten Bn = E.contract_new(raw_op(SVv.p, std::string{bw, 'j', 's'}, {Db, kB, 2}, {n, 2, 1}),
                                    op(QB, ew + "j"), ew + std::string{'s', bw});
            E.drop(QA);
            E.drop(QB);
            // 5. ungauge into the site tensors
            ungauge_site(E, An, ev + std::string{'s', bv}, Sp, zv, P.site[zv], lv, Dm);
            ungauge_site(E, Bn, ew + std::string{'s', bw}, Sp, zw, P.site[zw], lw, Dm);
            E.drop(An);
            E.drop(Bn);
        }
        TN_HIP(hipMemcpyAsync(eps_host, eps_d, (size_t)ng * 8, hipMemcpyDeviceToHost, E.s));
        E.sync();
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
}

}  // namespace tnb
