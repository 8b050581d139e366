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
// dropped, which makes the inverse a pseudo-inverse).  The gates of a group act
// on disjoint qubits and see the same messages, so they are independent: those
// with the same orientation and site shapes run as one batch.  Per gate (site
// v, site w sharing bond b of dimension D):
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

// Letters of a site tensor after gauging the legs in `done` (uppercase).
std::string letters(const bool done[5]) {
    std::string s;
    for (int k = 0; k < 5; ++k) s.push_back(done[k] ? GAUGED[k] : SLOT[k]);
    return s;
}

// The gates of one class (one group, same orientation, same shapes of both
// sites) go through every step together, as a batch over letter z: their
// sites, message roots and gate matrices are first gathered into contiguous
// [z][...] arrays by one table-driven copy, the results scattered back the
// same way.
struct GateClass {
    bool horiz;
    std::vector<int> da, db;  // site dims {p, u, l, d, r} of v and w
    std::vector<int> gates;   // indices into the gate list
};

// Gauge the three legs of the batched sites A [z][s][u][l][d][r] other than
// `bond` with the batched roots R[k] ([z][D_k][D_k], leg k): returns
// [z][G1][G2][G3][s][b] (G = gauged leg letters in slot order, b = SLOT[bond]).
Ten gauge_batch(Engine &E, const Ten &A, const Ten R[5], int bond, std::string &ext) {
    bool done[5] = {false, false, false, false, false};
    ext.clear();
    for (int k = 1; k <= 4; ++k)
        if (k != bond) ext.push_back(GAUGED[k]);
    Ten cur;
    bool have = false;
    int count = 0;
    try {
        for (int k = 1; k <= 4; ++k) {
            if (k == bond) continue;
            ++count;
            const std::string in = "z" + letters(done);
            done[k] = true;
            std::string out = "z" + letters(done);
            if (count == 3) out = "z" + ext + std::string{SLOT[0], SLOT[bond]};
            const Op src = have ? op(cur, in) : op(A, in);
            Ten nxt = E.contract_new(src, op(R[k], std::string{'z', SLOT[k], GAUGED[k]}), out);
            if (have) E.drop(cur);
            cur = nxt;
            have = true;
        }
    } catch (...) {
        if (have) E.drop(cur);
        throw;
    }
    return cur;
}

// Undo the gauge: T [z][in] (gauged legs uppercase), the batched pseudo-inverse
// roots applied leg by leg, the last product written to out [z][s][u][l][d][r].
void ungauge_batch(Engine &E, const Ten &T, const std::string &in, const Ten R[5], int bond, const Ten &out) {
    Ten cur;
    bool have = false;
    std::string cin = "z" + in;
    int count = 0;
    try {
        for (int k = 1; k <= 4; ++k) {
            if (k == bond) continue;
            ++count;
            std::string o = cin;
            o[o.find(GAUGED[k])] = SLOT[k];
            const Op src = have ? op(cur, cin) : op(T, cin);
            const Op Rk = op(R[k], std::string{'z', GAUGED[k], SLOT[k]});
            if (count == 3) {
                E.contract(src, Rk, op(out, "zsuldr"));
            } else {
                Ten nxt = E.contract_new(src, Rk, o);
                if (have) E.drop(cur);
                cur = nxt;
                have = true;
            }
            cin = o;
        }
    } catch (...) {
        if (have) E.drop(cur);
        throw;
    }
    if (have) E.drop(cur);
}

// Uploads a copy table and runs it; the host table must outlive the copy
// (kept in `keep` until the stream is synchronised).
void run_copies(Engine &E, std::vector<tnk::CopyBlock> &&tab, std::vector<std::vector<tnk::CopyBlock>> &keep,
                std::vector<void *> &raws) {
    if (tab.empty()) return;
    int64_t mx = 0;
    for (const auto &b : tab) mx = std::max<int64_t>(mx, b.rows * b.cols);
    keep.push_back(std::move(tab));
    const auto &t = keep.back();
    void *d = E.raw(t.size() * sizeof(tnk::CopyBlock));
    raws.push_back(d);
    TN_HIP(hipMemcpyAsync(d, t.data(), t.size() * sizeof(tnk::CopyBlock), hipMemcpyHostToDevice, E.s));
    TN_HIP(tnk::launch_copy_blocks(static_cast<const tnk::CopyBlock *>(d), (int)t.size(), mx, E.s));
}

}  // namespace

void simple_update(Engine &E, PepsDev &P, const std::vector<SuGate> &gates, const double *gmat, int gstride,
                   const SuOpts &o, double *eps_host, const void *msg_in, void *msg_out) {
    const int rows = P.rows, cols = P.cols, N = rows * cols;
    const int ng = (int)gates.size();
    if (ng == 0) return;
    int Dm = 1;
    for (const Ten &t : P.site)
        for (int k = 1; k <= 4; ++k) Dm = std::max(Dm, t.d[k]);
    if (Dm > 64) throw TnError(ST_UNSUPPORTED, "simple update: bonds above 64 (the pair SVD is at most 256 wide)");
    // gates of one group act on disjoint qubits (they are applied as one batch)
    {
        std::vector<int> seen((size_t)N, -1);
        int run = 0;
        for (int g = 0; g < ng; ++g) {
            if (g > 0 && gates[g].group != gates[g - 1].group) ++run;
            for (int z : {gates[g].r * cols + gates[g].c, gates[g].r2 * cols + gates[g].c2}) {
                if (seen[z] == run)
                    throw TnError(ST_INVALID, "gate " + std::to_string(g) + " shares a qubit with an earlier gate of its group");
                seen[z] = run;
            }
        }
    }
    const int nmat = gstride ? ng : 1;
    Ten Gd = E.make({nmat, 4, 4});
    Ten msg = E.make({N, 4, Dm, Dm});
    Ten Um = E.make({N * 4, Dm, Dm}), SVm = E.make({N * 4, Dm, Dm});
    Ten Sq = E.make({N * 4, Dm, Dm}), Sp = E.make({N * 4, Dm, Dm});
    int *kmsg = static_cast<int *>(E.raw((size_t)N * 4 * sizeof(int)));
    double *eps_d = static_cast<double *>(E.raw((size_t)ng * sizeof(double)));  // in processing order
    void *msg_ws = nullptr;
    if (const size_t wsb = tnk::svd_trunc_workspace_bytes(Dm, N * 4)) msg_ws = E.raw(wsb);
    std::vector<int> order;  // processing position -> gate index
    order.reserve((size_t)ng);
    std::vector<std::vector<tnk::CopyBlock>> keep;
    std::vector<void *> raws;
    std::vector<Ten> live;  // per-class tensors, dropped after each class
    auto drop_live = [&]() {
        for (Ten &t : live)
            if (t.p) E.drop(t);
        live.clear();
    };
    auto cleanup = [&]() {
        drop_live();
        E.drop(Gd); E.drop(msg); E.drop(Um); E.drop(SVm); E.drop(Sq); E.drop(Sp);
        E.unraw(kmsg); E.unraw(eps_d);
        if (msg_ws) E.unraw(msg_ws);
        for (void *p : raws) E.unraw(p);
        raws.clear();
    };
    auto keep_ten = [&](const std::vector<int> &d) -> Ten {
        live.push_back(E.make(d));
        return live.back();
    };
    try {
        TN_HIP(hipMemcpyAsync(Gd.p, gmat, (size_t)nmat * 16 * 16, hipMemcpyHostToDevice, E.s));
        bool first = true;
        if (msg_in) {  // continue from an earlier call's messages
            TN_HIP(hipMemcpyAsync(msg.p, msg_in, msg.bytes(), hipMemcpyDeviceToDevice, E.s));
            first = false;
        }
        for (int g0 = 0; g0 < ng;) {
            int g1 = g0;
            while (g1 < ng && gates[g1].group == gates[g0].group) ++g1;
            // BP messages of the current state, their roots and pseudo-inverse roots
            BpOpts bo;
            bo.max_sweeps = o.bp_max_sweeps;
            bo.tol = o.bp_tol;
            bo.loops = false;
            bo.messages = msg.p;
            bo.init_messages = first ? nullptr : msg.p;  // warm start from the previous group's messages
            BpResult br;
            bp_contract(E, P, bo, br);
            TN_HIP(tnk::launch_svd_trunc(static_cast<const double *>(msg.p), Dm, N * 4, 0.0, 0, Um.p, SVm.p, 16,
                                         kmsg, msg_ws, E.s));
            TN_HIP(tnk::launch_msg_roots(static_cast<const double *>(Um.p), static_cast<const double *>(SVm.p), Dm,
                                         N * 4, static_cast<double *>(Sq.p), static_cast<double *>(Sp.p), E.s));
            first = false;
            // classes of the group, in order of first appearance
            std::vector<GateClass> cls;
            for (int g = g0; g < g1; ++g) {
                const SuGate &q = gates[g];
                const bool horiz = q.r2 == q.r;
                const Ten &A = P.site[(size_t)q.r * cols + q.c], &B = P.site[(size_t)q.r2 * cols + q.c2];
                auto it = std::find_if(cls.begin(), cls.end(), [&](const GateClass &c) {
                    return c.horiz == horiz && c.da == A.d && c.db == B.d;
                });
                if (it == cls.end()) {
                    cls.push_back(GateClass{horiz, A.d, B.d, {}});
                    it = cls.end() - 1;
                }
                it->gates.push_back(g);
            }
            for (const GateClass &C : cls) {
                const int G = (int)C.gates.size();
                const int lv = C.horiz ? 4 : 3, lw = C.horiz ? 2 : 1;
                const int Db = C.da[lv];
                const int64_t na = Ten{nullptr, C.da}.numel(), nb = Ten{nullptr, C.db}.numel();
                // 0. gather sites, roots (square and pseudo-inverse) and gate matrices
                std::vector<int> bda = C.da, bdb = C.db;
                bda.insert(bda.begin(), G);
                bdb.insert(bdb.begin(), G);
                Ten Ab = keep_ten(bda), Bb = keep_ten(bdb);
                Ten RqA[5], RpA[5], RqB[5], RpB[5];
                for (int k = 1; k <= 4; ++k) {
                    if (k != lv) { RqA[k] = keep_ten({G, C.da[k], C.da[k]}); RpA[k] = keep_ten({G, C.da[k], C.da[k]}); }
                    if (k != lw) { RqB[k] = keep_ten({G, C.db[k], C.db[k]}); RpB[k] = keep_ten({G, C.db[k], C.db[k]}); }
                }
                Ten Gb;
                if (gstride) Gb = keep_ten({G, 16});
                std::vector<tnk::CopyBlock> tab;
                auto root_src = [&](const Ten &roots, int z, int k) {
                    return static_cast<const char *>(roots.p) + (((size_t)z * 4 + (k - 1)) * Dm * Dm) * 16;
                };
                for (int i = 0; i < G; ++i) {
                    const SuGate &q = gates[C.gates[(size_t)i]];
                    const int zv = q.r * cols + q.c, zw = q.r2 * cols + q.c2;
                    tab.push_back({P.site[(size_t)zv].p, static_cast<char *>(Ab.p) + (size_t)i * na * 16, 1, na, 0});
                    tab.push_back({P.site[(size_t)zw].p, static_cast<char *>(Bb.p) + (size_t)i * nb * 16, 1, nb, 0});
                    for (int k = 1; k <= 4; ++k) {
                        if (k != lv) {
                            const int64_t Dk = C.da[k];
                            tab.push_back({root_src(Sq, zv, k), static_cast<char *>(RqA[k].p) + (size_t)i * Dk * Dk * 16,
                                           Dk, Dk, Dm});
                            tab.push_back({root_src(Sp, zv, k), static_cast<char *>(RpA[k].p) + (size_t)i * Dk * Dk * 16,
                                           Dk, Dk, Dm});
                        }
                        if (k != lw) {
                            const int64_t Dk = C.db[k];
                            tab.push_back({root_src(Sq, zw, k), static_cast<char *>(RqB[k].p) + (size_t)i * Dk * Dk * 16,
                                           Dk, Dk, Dm});
                            tab.push_back({root_src(Sp, zw, k), static_cast<char *>(RpB[k].p) + (size_t)i * Dk * Dk * 16,
                                           Dk, Dk, Dm});
                        }
                    }
                    if (gstride)
                        tab.push_back({static_cast<const char *>(Gd.p) + (size_t)C.gates[(size_t)i] * 16 * 16,
                                       static_cast<char *>(Gb.p) + (size_t)i * 16 * 16, 1, 16, 0});
                }
                run_copies(E, std::move(tab), keep, raws);
                // 1. gauge, ordered [z][other legs][phys][bond]
                std::string ev, ew;
                Ten Ag = gauge_batch(E, Ab, RqA, lv, ev);
                Ten Bg = gauge_batch(E, Bb, RqB, lw, ew);
                // 2. QR of (other legs) x (phys, bond), batched over z
                const std::vector<int> agd = Ag.d, bgd = Bg.d;
                Ag.d = {G, agd[1], agd[2], agd[3], agd[4] * agd[5]};
                Bg.d = {G, bgd[1], bgd[2], bgd[3], bgd[4] * bgd[5]};
                Ten QA, RA, QB, RB;
                qr_left(E, Ag, 1, QA, &RA);
                qr_left(E, Bg, 1, QB, &RB);
                E.drop(Ag);
                E.drop(Bg);
                live.push_back(QA);
                live.push_back(QB);
                const int kA = RA.d[1], kB = RB.d[1];
                RA.d = {G, kA, 2, Db};
                RB.d = {G, kB, 2, Db};
                // 3. theta through the gate, into zero-padded squares whose side
                // holds both factors' rows and the bond's D columns
                const int n = std::max(std::max(2 * kA, 2 * kB), Db);
                const int64_t nn = (int64_t)n * n;
                Ten T1 = E.contract_new(op(RA, "zisb"), op(RB, "zjtb"), "zisjt");
                E.drop(RA);
                E.drop(RB);
                Ten M = keep_ten({G, (int)nn}), Uv = keep_ten({G, (int)nn}), SVv = keep_ten({G, (int)nn});
                TN_HIP(tnk::launch_fill(M.p, 16, G * nn, 0.0, 0.0, E.s));
                const Op gop = gstride ? raw_op(Gb.p, "zSTst", {G, 2, 2, 2, 2}, {16, 8, 4, 2, 1})
                                       : raw_op(Gd.p, "zSTst", {G, 2, 2, 2, 2}, {0, 8, 4, 2, 1});
                E.contract(op(T1, "zisjt"), gop, raw_op(M.p, "ziSjT", {G, kA, 2, kB, 2}, {nn, 2LL * n, n, 2, 1}));
                E.drop(T1);
                E.normalise(M.p, 16, nn, G, nn, nullptr, false, nullptr);
                // 4. truncated SVDs, balanced factors
                int *kg = static_cast<int *>(E.raw((size_t)G * sizeof(int)));
                raws.push_back(kg);
                void *ws = nullptr;
                if (const size_t wsb = tnk::svd_trunc_workspace_bytes(n, G)) {
                    ws = E.raw(wsb);
                    raws.push_back(ws);
                }
                TN_HIP(tnk::launch_svd_trunc(static_cast<const double *>(M.p), n, G, 0.0, 0, Uv.p, SVv.p, 16, kg, ws,
                                             E.s, Db, eps_d + order.size()));
                TN_HIP(tnk::launch_split_sqrt(static_cast<double *>(Uv.p), static_cast<double *>(SVv.p), n, G, E.s));
                for (int g : C.gates) order.push_back(g);
                const char bv = SLOT[lv], bw = SLOT[lw];
                // v: [z][ev][s][b] = sum_i Q_A[z][ev][i] U[z][(i s)][b]
                Ten An = E.contract_new(op(QA, "z" + ev + "i"),
                                        raw_op(Uv.p, std::string{'z', 'i', 's', bv}, {G, kA, 2, Db}, {nn, 2LL * n, n, 1}),
                                        "z" + ev + std::string{'s', bv});
                // w: [z][ew][t][b] = sum_j SV[z][b][(j t)] Q_B[z][ew][j]
                Ten Bn = E.contract_new(raw_op(SVv.p, std::string{'z', bw, 'j', 's'}, {G, Db, kB, 2}, {nn, n, 2, 1}),
                                        op(QB, "z" + ew + "j"), "z" + ew + std::string{'s', bw});
                // 5. ungauge into batched outputs, scattered to the site tensors
                Ten Ao = keep_ten(bda), Bo = keep_ten(bdb);
                ungauge_batch(E, An, ev + std::string{'s', bv}, RpA, lv, Ao);
                ungauge_batch(E, Bn, ew + std::string{'s', bw}, RpB, lw, Bo);
                E.drop(An);
                E.drop(Bn);
                std::vector<tnk::CopyBlock> sc;
                for (int i = 0; i < G; ++i) {
                    const SuGate &q = gates[C.gates[(size_t)i]];
                    sc.push_back({static_cast<const char *>(Ao.p) + (size_t)i * na * 16,
                                  P.site[(size_t)q.r * cols + q.c].p, 1, na, 0});
                    sc.push_back({static_cast<const char *>(Bo.p) + (size_t)i * nb * 16,
                                  P.site[(size_t)q.r2 * cols + q.c2].p, 1, nb, 0});
                }
                run_copies(E, std::move(sc), keep, raws);
                drop_live();
            }
            // the tables' host copies may go once the stream has passed them
            E.sync();
            keep.clear();
            for (void *p : raws) E.unraw(p);
            raws.clear();
            g0 = g1;
        }
        if (msg_out) TN_HIP(hipMemcpyAsync(msg_out, msg.p, msg.bytes(), hipMemcpyDeviceToDevice, E.s));
        std::vector<double> tmp((size_t)ng);
        TN_HIP(hipMemcpyAsync(tmp.data(), eps_d, (size_t)ng * 8, hipMemcpyDeviceToHost, E.s));
        E.sync();
        for (int j = 0; j < ng; ++j) eps_host[order[(size_t)j]] = tmp[(size_t)j];
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
}

}  // namespace tnb
