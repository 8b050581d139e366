// Belief propagation on the norm network <psi|psi> and the loop BP error
// (Methods, "Quantum Circuit Simulation" -- message tensors by BP -- and "The
// Boundary Matrix Product State Method" -- BP contraction, Eqs. avBPError and
// loopBPerror; Appendix, "Applying Gates to a Tensor Network State" -- the
// message update and its normalisation -- and "Computing the BP Error").
//
// Every site other than a dummy (a scalar without bonds, which only
// contributes Z_v = 1 and e0 e0^T messages) takes part; the sites are grouped
// by shape and each group's contractions run on its own dimensions (a site
// with three bonds costs D^4, not Dm^5, per message).  Messages are stored
// padded to the largest bond Dm:
// msg[z][leg][k][k'] (into site z through leg, ket index k, bra index k'),
// e0 e0^T on legs without a bond, so padded entries never contribute.  A
// parallel sweep computes, for each of the four legs, the message every site
// sends through it -- the pair (A, conj A) closed with the site's other three
// incoming messages, three batched contractions over all sites and one with
// conj(A) -- then k_bp_update takes each one's Hermitian part, normalises it to
// unit Frobenius norm and stores it as the neighbour's incoming message.
// FP64 throughout.
#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <string>
#include <vector>

#include "tn_core.hpp"

namespace tnb {

namespace {

constexpr int NLEG = 4;  // 0 up, 1 left, 2 down, 3 right (axes 1..4 of a site tensor)
const char KET[NLEG] = {'a', 'b', 'c', 'd'};
const char BRA[NLEG] = {'e', 'f', 'g', 'h'};
const int DR[NLEG] = {-1, 0, 1, 0}, DC[NLEG] = {0, -1, 0, 1};

// The sites of one shape: their tensors stored unpadded, [count][p][u][l][d][r],
// occupying active indices start .. start + count - 1.
struct SiteClass {
    int start = 0, count = 0;
    int dims[5] = {1, 1, 1, 1, 1};
    Ten A;
};

// View of one class's incoming messages of one leg: the D x D blocks of
// msg[z][leg][k][k'] for z in the class.
Op msg_op(const Ten &msg, const SiteClass &c, int leg, int Dm) {
    Op o;
    o.p = static_cast<const char *>(msg.p) + ((size_t)c.start * NLEG + leg) * Dm * Dm * msg.esz;
    o.esz = msg.esz;
    o.idx = std::string("z") + KET[leg] + BRA[leg];
    o.dims = {c.count, c.dims[leg + 1], c.dims[leg + 1]};
    o.str = {(int64_t)NLEG * Dm * Dm, Dm, 1};
    return o;
}

Op class_op(const SiteClass &c, const std::string &idx, bool conj) {
    Op o;
    o.p = c.A.p;
    o.esz = c.A.esz;
    o.idx = idx;
    o.dims = {c.count, c.dims[0], c.dims[1], c.dims[2], c.dims[3], c.dims[4]};
    o.str.assign(6, 1);
    for (int i = 4; i >= 0; --i) o.str[(size_t)i] = o.str[(size_t)i + 1] * o.dims[(size_t)i + 1];
    o.conj = conj;
    return o;
}

// The pair (A, conj A) of every site of the class with the incoming messages
// on all legs not in `keep` contracted; result [z] + (ket, bra) letters of the
// kept legs in order, written through `out` (the caller's view of the class's
// blocks; every dimension is the site's own, nothing is padded).
void pair_closed(Engine &E, const SiteClass &c, const Ten &msg, const std::vector<int> &keep, const Op &out,
                 int Dm) {
    std::string cur = "zsabcd";
    Ten t;  // current intermediate (empty: A itself)
    for (int leg = 0; leg < NLEG; ++leg) {
        if (std::find(keep.begin(), keep.end(), leg) != keep.end()) continue;
        std::string nxt;
        for (char ch : cur)
            if (ch != KET[leg]) nxt += ch;
        nxt += BRA[leg];
        Ten r = E.contract_new(t.p ? op(t, cur) : class_op(c, cur, false), msg_op(msg, c, leg, Dm), nxt);
        if (t.p) E.drop(t);
        t = r;
        cur = nxt;
    }
    // close with conj(A) over s and the bra legs of the contracted legs
    E.contract(op(t, cur), class_op(c, "zsefgh", true), out);
    E.drop(t);
}

// Contracts the incoming messages of `legs` into the intermediate `t`
// (letters `cur`; t empty = the class's site tensors A themselves): each
// message replaces a ket letter by its bra letter.
Ten with_messages(Engine &E, const SiteClass &c, const Ten &msg, const Ten &t, std::string &cur,
                  const std::vector<int> &legs, int Dm) {
    Ten r = t;
    bool own = false;
    try {
        for (int leg : legs) {
            std::string nxt;
            for (char ch : cur)
                if (ch != KET[leg]) nxt += ch;
            nxt += BRA[leg];
            Ten x = E.contract_new(r.p ? op(r, cur) : class_op(c, cur, false), msg_op(msg, c, leg, Dm), nxt);
            if (own) E.drop(r);
            r = x;
            own = true;
            cur = nxt;
        }
    } catch (...) {
        if (own) E.drop(r);
        throw;
    }
    return r;
}

// The four outgoing messages of every site of the class into out_op(leg):
// the same values as pair_closed with keep = {leg} for each leg, from shared
// partial products (A with the messages of legs 2 and 3 serves the outputs
// of legs 0 and 1, A with those of legs 0 and 1 the outputs of legs 2 and 3):
// 12 contractions instead of 16.
template <typename OutOp>
void all_outgoing(Engine &E, const SiteClass &c, const Ten &msg, int Dm, OutOp out_op) {
    const int pairs[2][2] = {{2, 3}, {0, 1}};  // legs contracted first; the outputs are the other two
    for (const auto &pr : pairs) {
        std::string base = "zsabcd";
        Ten X = with_messages(E, c, msg, Ten{}, base, {pr[0], pr[1]}, Dm);
        const int o0 = pr[0] == 2 ? 0 : 2;
        try {
            for (int q = 0; q < 2; ++q) {
                const int keep = o0 + q, other = o0 + 1 - q;
                std::string cur = base;
                Ten Y = with_messages(E, c, msg, X, cur, {other}, Dm);
                try {
                    E.contract(op(Y, cur), class_op(c, "zsefgh", true), out_op(keep, c));
                } catch (...) {
                    E.drop(Y);
                    throw;
                }
                E.drop(Y);
            }
        } catch (...) {
            E.drop(X);
            throw;
        }
        E.drop(X);
    }
}

// Faces of the planar grid embedding (grid cells merged across absent bonds,
// those not connected to the outside), each as the cycle of its boundary
// sites: (site, in_leg, out_leg) in walk order, starting at the smallest site
// (row-major) and stepping first to its smaller boundary neighbour.
struct LoopSite { int z, lin, lout; };
std::vector<std::vector<LoopSite>> faces(const PepsDev &P) {
    const int rows = P.rows, cols = P.cols;
    auto hb = [&](int r, int c) { return c + 1 < cols && P.at(r, c).d[4] > 1; };
    auto vb = [&](int r, int c) { return r + 1 < rows && P.at(r, c).d[3] > 1; };
    std::vector<std::vector<LoopSite>> loops;
    const int nr = rows - 1, nc = cols - 1;
    if (nr <= 0 || nc <= 0) return loops;
    const int OUT = nr * nc;
    std::vector<int> parent(OUT + 1);
    std::iota(parent.begin(), parent.end(), 0);
    auto find = [&](int x) {
        while (parent[x] != x) x = parent[x] = parent[parent[x]];
        return x;
    };
    auto cell = [&](int i, int j) { return (i >= 0 && i < nr && j >= 0 && j < nc) ? i * nc + j : OUT; };
    auto unite = [&](int a, int b) { parent[find(a)] = find(b); };
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nc; ++j) {
            if (!hb(i, j)) unite(cell(i, j), cell(i - 1, j));
            if (!hb(i + 1, j)) unite(cell(i, j), cell(i + 1, j));
            if (!vb(i, j)) unite(cell(i, j), cell(i, j - 1));
            if (!vb(i, j + 1)) unite(cell(i, j), cell(i, j + 1));
        }
    std::map<int, std::vector<std::pair<int, int>>> groups;
    for (int i = 0; i < nr; ++i)
        for (int j = 0; j < nc; ++j) {
            const int root = find(cell(i, j));
            if (root != find(OUT)) groups[root].push_back({i, j});
        }
    for (auto &kv : groups) {
        std::vector<int> in(nr * nc, 0);
        for (auto &ij : kv.second) in[ij.first * nc + ij.second] = 1;
        auto inside = [&](int i, int j) { return i >= 0 && i < nr && j >= 0 && j < nc && in[i * nc + j]; };
        std::map<int, std::vector<int>> adj;  // site -> boundary neighbours
        auto add = [&](int r1, int c1, int r2, int c2) {
            adj[r1 * cols + c1].push_back(r2 * cols + c2);
            adj[r2 * cols + c2].push_back(r1 * cols + c1);
        };
        for (auto &ij : kv.second) {
            const int i = ij.first, j = ij.second;
            if (!inside(i - 1, j)) add(i, j, i, j + 1);
            if (!inside(i + 1, j)) add(i + 1, j, i + 1, j + 1);
            if (!inside(i, j - 1)) add(i, j, i + 1, j);
            if (!inside(i, j + 1)) add(i, j + 1, i + 1, j + 1);
        }
        for (auto &a : adj)
            if (a.second.size() != 2) throw TnError(ST_UNSUPPORTED, "a face of the lattice is not a simple cycle");
        const int start = adj.begin()->first;
        std::vector<int> cyc = {start};
        int prev = -1, cur = start;
        std::vector<int> &s0 = adj[start];
        int nxt = std::min(s0[0], s0[1]);
        while (nxt != start) {
            cyc.push_back(nxt);
            prev = cur;
            cur = nxt;
            const std::vector<int> &a = adj[cur];
            nxt = a[0] != prev ? a[0] : a[1];
        }
        auto leg_to = [&](int a, int b) {
            const int dr = b / cols - a / cols, dc = b % cols - a % cols;
            for (int l = 0; l < NLEG; ++l)
                if (DR[l] == dr && DC[l] == dc) return l;
            throw TnError(ST_SHAPE, "face walk between non-neighbours");
        };
        const int L = (int)cyc.size();
        std::vector<LoopSite> lp(L);
        for (int k = 0; k < L; ++k)
            lp[k] = {cyc[k], leg_to(cyc[k], cyc[(k + L - 1) % L]), leg_to(cyc[k], cyc[(k + 1) % L])};
        loops.push_back(lp);
    }
    std::sort(loops.begin(), loops.end(),
              [](const std::vector<LoopSite> &a, const std::vector<LoopSite> &b) { return a[0].z < b[0].z; });
    return loops;
}

}  // namespace

void bp_contract(Engine &E, const PepsDev &P, const BpOpts &o, BpResult &res) {
    const int rows = P.rows, cols = P.cols, NG = rows * cols;
    int Dm = 1;
    for (const Ten &t : P.site)
        for (int k = 1; k <= 4; ++k) Dm = std::max(Dm, t.d[k]);
    const int n2 = Dm * Dm;
    // the sites that take part: every grid position except dummies (a scalar
    // tensor with no bond: its messages are e0 e0^T and its Z_v is 1), grouped
    // by shape so that each group's contractions run on its own dimensions
    std::map<std::vector<int>, std::vector<int>> shapes;
    for (int z = 0; z < NG; ++z) {
        const Ten &t = P.site[(size_t)z];
        if (t.numel() > 1) shapes[t.d].push_back(z);
    }
    std::vector<int> act, aidx((size_t)NG, -1);
    std::vector<SiteClass> cls;
    for (auto &kv : shapes) {
        SiteClass c;
        c.start = (int)act.size();
        c.count = (int)kv.second.size();
        for (int i = 0; i < 5; ++i) c.dims[i] = kv.first[(size_t)i];
        for (int z : kv.second) {
            aidx[(size_t)z] = (int)act.size();
            act.push_back(z);
        }
        cls.push_back(c);
    }
    const int N = (int)act.size();
    if (N == 0) throw TnError(ST_INVALID, "belief propagation: the state has no site with a bond or a qubit");
    for (auto &c : cls) {
        c.A = E.make({c.count, c.dims[0], c.dims[1], c.dims[2], c.dims[3], c.dims[4]});
        const size_t bytes = (size_t)c.dims[0] * c.dims[1] * c.dims[2] * c.dims[3] * c.dims[4] * 16;
        for (int i = 0; i < c.count; ++i) {
            const Ten &t = P.site[(size_t)act[(size_t)c.start + i]];
            if (t.esz != 16) throw TnError(ST_INVALID, "belief propagation runs on complex128 site tensors");
            TN_HIP(hipMemcpyAsync(static_cast<char *>(c.A.p) + (size_t)i * bytes, t.p, bytes,
                                  hipMemcpyDeviceToDevice, E.s));
        }
    }
    // neighbour table and initial messages: identity / sqrt(D) on bonds, e0 e0^T elsewhere
    std::vector<int> hn((size_t)N * NLEG, -1);
    std::vector<double> hm((size_t)N * NLEG * n2 * 2, 0.0);
    for (int i = 0; i < N; ++i) {
        const int r = act[i] / cols, c = act[i] % cols;
        for (int leg = 0; leg < NLEG; ++leg) {
            const int D = P.at(r, c).d[leg + 1];
            const int r2 = r + DR[leg], c2 = c + DC[leg];
            const bool bond = D > 1 && r2 >= 0 && r2 < rows && c2 >= 0 && c2 < cols;
            double *m = hm.data() + ((size_t)i * NLEG + leg) * n2 * 2;
            if (bond) {
                const int j = aidx[(size_t)r2 * cols + c2];
                if (j < 0) throw TnError(ST_SHAPE, "belief propagation: a bond leads to a dummy site");
                hn[(size_t)i * NLEG + leg] = j;
                for (int k = 0; k < D; ++k) m[(k * Dm + k) * 2] = 1.0 / std::sqrt((double)D);
            } else {
                m[0] = 1.0;
            }
        }
    }
    Ten msg = E.make({N, NLEG, Dm, Dm});
    int *nbr = static_cast<int *>(E.raw(hn.size() * sizeof(int)));
    Ten out = E.make({NLEG, N, Dm, Dm});
    double *dmax = static_cast<double *>(E.raw((size_t)N * NLEG * 8));
    double *dscal = static_cast<double *>(E.raw(64));
    const size_t site_msgs = (size_t)NLEG * n2 * 16;  // bytes of one site's four messages
    auto cleanup = [&]() {
        for (auto &c : cls)
            if (c.A.p) E.drop(c.A);
        E.drop(msg);
        E.drop(out);
        E.unraw(nbr);
        E.unraw(dmax);
        E.unraw(dscal);
    };
    try {
        if (o.init_messages) {  // grid layout [NG][4][Dm][Dm]: the active sites' blocks
            for (int i = 0; i < N; ++i)
                TN_HIP(hipMemcpyAsync(static_cast<char *>(msg.p) + (size_t)i * site_msgs,
                                      static_cast<const char *>(o.init_messages) + (size_t)act[i] * site_msgs,
                                      site_msgs, hipMemcpyDeviceToDevice, E.s));
        } else {
            TN_HIP(hipMemcpyAsync(msg.p, hm.data(), hm.size() * 8, hipMemcpyHostToDevice, E.s));
        }
        TN_HIP(hipMemcpyAsync(nbr, hn.data(), hn.size() * sizeof(int), hipMemcpyHostToDevice, E.s));
        // the sweeps write each site's own D x D block of its outgoing messages
        TN_HIP(tnk::launch_fill(out.p, out.esz, out.numel(), 0.0, 0.0, E.s));
        E.sync();  // the host arrays above are released on return
        auto out_op = [&](int leg, const SiteClass &c) {
            Op q;
            q.p = static_cast<char *>(out.p) + ((size_t)leg * N + c.start) * n2 * out.esz;
            q.esz = out.esz;
            q.idx = std::string("z") + KET[leg] + BRA[leg];
            q.dims = {c.count, c.dims[leg + 1], c.dims[leg + 1]};
            q.str = {(int64_t)n2, Dm, 1};
            return q;
        };
        double delta = INFINITY;
        int sweep = 0;
        while (sweep < o.max_sweeps) {
            for (const auto &c : cls) all_outgoing(E, c, msg, Dm, out_op);
            TN_HIP(tnk::launch_bp_update(out.p, msg.p, nbr, N, Dm, dmax, dscal, E.s));
            ++sweep;
            if (sweep % 4 == 0 || sweep == o.max_sweeps) {
                TN_HIP(hipMemcpyAsync(&delta, dscal, 8, hipMemcpyDeviceToHost, E.s));
                E.sync();
                if (!(delta < INFINITY)) throw TnError(ST_NUMERIC, "BP message vanished or overflowed");
                if (delta < o.tol) break;
            }
        }
        res.sweeps = sweep;
        res.delta = delta;
        // Z_BP from the final messages
        for (const auto &c : cls) pair_closed(E, c, msg, {3}, out_op(3, c), Dm);
        double *zv = static_cast<double *>(E.raw((size_t)N * 16));
        double *ze = static_cast<double *>(E.raw((size_t)N * 32));
        TN_HIP(tnk::launch_bp_free_energy(static_cast<char *>(out.p) + (size_t)3 * N * n2 * 16, msg.p, nbr, N, Dm,
                                          zv, ze, dscal, E.s));
        double h2[2];
        TN_HIP(hipMemcpyAsync(h2, dscal, 16, hipMemcpyDeviceToHost, E.s));
        E.sync();
        E.unraw(zv);
        E.unraw(ze);
        res.log_abs = h2[0];
        res.arg = h2[1];
        if (o.messages) {
            // grid layout [NG][4][Dm][Dm]: dummies hold e0 e0^T on every leg
            std::vector<double> dm((size_t)NG * NLEG * n2 * 2, 0.0);
            for (size_t q = 0; q < (size_t)NG * NLEG; ++q) dm[q * n2 * 2] = 1.0;
            TN_HIP(hipMemcpyAsync(o.messages, dm.data(), dm.size() * 8, hipMemcpyHostToDevice, E.s));
            for (int i = 0; i < N; ++i)
                TN_HIP(hipMemcpyAsync(static_cast<char *>(o.messages) + (size_t)act[i] * site_msgs,
                                      static_cast<const char *>(msg.p) + (size_t)i * site_msgs, site_msgs,
                                      hipMemcpyDeviceToDevice, E.s));
            E.sync();  // dm is released on return
        }
        // loop BP error
        res.eps.clear();
        res.eps_mean = 0.0;
        res.eig_info = 0;
        if (o.loops) {
            const std::vector<std::vector<LoopSite>> loops = faces(P);
            if (!loops.empty()) {
                if (n2 > tnk::BP_EIG_NMAX)
                    throw TnError(ST_UNSUPPORTED, "loop BP error supports bonds up to " +
                                                      std::to_string((int)std::sqrt((double)tnk::BP_EIG_NMAX)));
                // pair tensors of every site for the leg pairs the loops use: [z][a][a'][b][b'], a < b
                int pid[NLEG][NLEG];
                for (auto &x : pid)
                    for (int &y : x) y = -1;
                std::vector<std::pair<int, int>> pairs;
                for (auto &lp : loops)
                    for (auto &s : lp) {
                        const int a = std::min(s.lin, s.lout), b = std::max(s.lin, s.lout);
                        if (pid[a][b] < 0) {
                            pid[a][b] = (int)pairs.size();
                            pairs.push_back({a, b});
                        }
                    }
                Ten pt = E.make({(int)pairs.size(), N, Dm, Dm, Dm, Dm});
                TN_HIP(tnk::launch_fill(pt.p, pt.esz, pt.numel(), 0.0, 0.0, E.s));
                const size_t pstride = (size_t)N * n2 * n2;
                for (size_t k = 0; k < pairs.size(); ++k)
                    for (const auto &c : cls) {
                        const int a = pairs[k].first, b = pairs[k].second;
                        Op q;
                        q.p = static_cast<char *>(pt.p) + (k * pstride + (size_t)c.start * n2 * n2) * 16;
                        q.esz = 16;
                        q.idx = std::string("z") + KET[a] + BRA[a] + KET[b] + BRA[b];
                        q.dims = {c.count, c.dims[a + 1], c.dims[a + 1], c.dims[b + 1], c.dims[b + 1]};
                        q.str = {(int64_t)n2 * n2, (int64_t)Dm * n2, n2, Dm, 1};
                        pair_closed(E, c, msg, {a, b}, q, Dm);
                    }
                // loops grouped by length: gather [loop][k] matrices, multiply along the walk
                std::map<int, std::vector<int>> bylen;
                for (int i = 0; i < (int)loops.size(); ++i) bylen[(int)loops[i].size()].push_back(i);
                std::vector<double> heps(loops.size(), 0.0);
                std::vector<int> hinfo(loops.size(), 0);
                for (auto &g : bylen) {
                    const int L = g.first, nl = (int)g.second.size();
                    std::vector<int64_t> hoff((size_t)nl * L);
                    std::vector<int> htr((size_t)nl * L);
                    for (int i = 0; i < nl; ++i)
                        for (int k = 0; k < L; ++k) {
                            const LoopSite &s = loops[g.second[i]][k];
                            const int a = std::min(s.lin, s.lout), b = std::max(s.lin, s.lout);
                            hoff[(size_t)i * L + k] = (int64_t)pid[a][b] * pstride + (int64_t)aidx[(size_t)s.z] * n2 * n2;
                            htr[(size_t)i * L + k] = s.lin == a ? 0 : 1;  // walk enters through the larger leg
                        }
                    int64_t *doff = static_cast<int64_t *>(E.raw(hoff.size() * 8));
                    int *dtr = static_cast<int *>(E.raw(htr.size() * 4));
                    Ten mats = E.make({nl, L, n2, n2});
                    Ten X = E.make({nl, n2, n2}), Y = E.make({nl, n2, n2});
                    double *deps = static_cast<double *>(E.raw((size_t)nl * 8));
                    int *dinfo = static_cast<int *>(E.raw((size_t)nl * 4));
                    double *lam = static_cast<double *>(E.raw((size_t)nl * n2 * 16));
                    TN_HIP(hipMemcpyAsync(doff, hoff.data(), hoff.size() * 8, hipMemcpyHostToDevice, E.s));
                    TN_HIP(hipMemcpyAsync(dtr, htr.data(), htr.size() * 4, hipMemcpyHostToDevice, E.s));
                    TN_HIP(tnk::launch_gather_mats(pt.p, doff, dtr, nl * L, n2, mats.p, E.s));
                    auto mat_op = [&](int k, const std::string &idx) {
                        Op q;
                        q.p = static_cast<char *>(mats.p) + (size_t)k * n2 * n2 * 16;
                        q.esz = 16;
                        q.idx = idx;
                        q.dims = {nl, n2, n2};
                        q.str = {(int64_t)L * n2 * n2, n2, 1};
                        return q;
                    };
                    // X = M_0 M_1 ... M_{L-1}
                    E.contract(mat_op(0, "xij"), mat_op(1, "xjk"), op(X, "xik"));
                    for (int k = 2; k < L; ++k) {
                        E.contract(op(X, "xij"), mat_op(k, "xjk"), op(Y, "xik"));
                        std::swap(X, Y);
                    }
                    TN_HIP(tnk::launch_eig(X.p, n2, nl, lam, deps, dinfo, E.s));
                    std::vector<double> e(nl);
                    std::vector<int> inf(nl);
                    TN_HIP(hipMemcpyAsync(e.data(), deps, (size_t)nl * 8, hipMemcpyDeviceToHost, E.s));
                    TN_HIP(hipMemcpyAsync(inf.data(), dinfo, (size_t)nl * 4, hipMemcpyDeviceToHost, E.s));
                    E.sync();
                    for (int i = 0; i < nl; ++i) {
                        heps[g.second[i]] = e[i];
                        hinfo[g.second[i]] = inf[i];
                    }
                    E.unraw(doff);
                    E.unraw(dtr);
                    E.unraw(deps);
                    E.unraw(dinfo);
                    E.unraw(lam);
                    E.drop(mats);
                    E.drop(X);
                    E.drop(Y);
                }
                E.drop(pt);
                res.eps = heps;
                double s = 0.0;
                for (double v : heps) s += v;
                res.eps_mean = s / (double)heps.size();
                for (int v : hinfo) res.eig_info |= v;
            }
        }
    } catch (...) {
        cleanup();
        throw;
    }
    cleanup();
}

}  // namespace tnb
